// Plain structs shared by the host runtime and the kernels: grid geometry,
// physical constants in the working precision, and views of the particle
// arrays in the workspace.
#pragma once

#include <stdint.h>

namespace mpm {

enum { WALL_SLIP = 0, WALL_STICK = 1, WALL_COULOMB = 2 };
enum { MAT_FLUID = 0, MAT_SAND = 1, MAT_ELASTIC = 2 };

// Tile-padded node grid.  Node stored index I = i + G for physical node i
// (at i*h).  A tile is T cells per axis (64 cells); its P2G/G2P node block
// is T+2 nodes per axis starting at the tile origin.
struct Geo {
    int dim;
    int T;              // tile edge in cells
    int n[3];           // cells per axis (1 for unused axes)
    int G;              // ghost layers
    int bmax[3];        // largest valid base + G  (= n + 2G)
    int ntile[3];       // tiles per axis (1 for unused axes)
    int ntiles;
    int nd[3];          // nodes per axis of the tile-padded grid
    long long NN;       // nodes in the tile-padded grid
    int box[3];         // dense node box n + 1 + 2G (the ABI's grid layout)
};

template <class T>
struct Phys {
    T h, inv, Dinv, dt, mass, vol0;
    T g[3];
    T ext[3];           // domain extent n*h
    T lam, mu;          // Lame constants (sand / elastic)
    T cone_coef;        // (d lam + 2 mu) / (2 mu) * alpha
    T k_over_gamma, gamma;
    int material;
    int wall_mode[6];
    T wall_mu[6];
    const T* floor_mu;  // per floor node, or null
    int floor_stride;   // floor row length (box[0])
    int keep_grid;
};

// One buffer of particle state, component-major with stride cap.
//   x[D], v[D], C[D*D], then sand: G[D*D] (= F_e - I), S[D(D+1)/2]
//                            fluid: dJ[1] (= J - 1), S[1]
template <class T>
struct PView {
    T* x;
    T* v;
    T* C;
    T* G;      // or dJ
    T* S;
    int32_t* pid;
    long long cap;
};

struct ActiveTile {
    int tile, off, cnt, pad;
};

}  // namespace mpm
