// Plain structs shared by the host runtime and the kernels: grid geometry,
// physical constants in the working precision, and views of the particle
// arrays in the workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

enum { WALL_SLIP = 0, WALL_STICK = 1, WALL_COULOMB = 2 };
// Kernel materials.  FLUID carries J and one isotropic stress value; the
// others carry the full symmetric stress cache, and either F_e - I (SAND,
// ELASTIC: Hencky strain) or J (VFLUID: viscous fluid; JAUMANN: hypoelastic
// Drucker-Prager).
enum { MAT_FLUID = 0, MAT_SAND = 1, MAT_ELASTIC = 2, MAT_VFLUID = 3, MAT_JAUMANN = 4 };
// Grid-to-particle transfers (App. B).
enum { XF_APIC = 0, XF_PIC = 1, XF_FLIP = 2, XF_TPIC = 3 };
constexpr int kMaxObstacles = 4;

__host__ __device__ constexpr bool mat_has_F(int mat) { return mat == MAT_SAND || mat == MAT_ELASTIC; }
__host__ __device__ constexpr bool mat_iso_stress(int mat) { return mat == MAT_FLUID; }

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
    int xfer;           // XF_*
    T flip_alpha;       // FLIP share of the FLIP/PIC blend
    T visc;             // fluid dynamic viscosity
    // hypoelastic Drucker-Prager (App. A): bulk modulus, q_phi, k_phi,
    // q_psi, sigma^t, tau^P = k_phi - q_phi sigma^t, alpha^P, elastic band
    T jK, jq_phi, jk_phi, jq_psi, jst, jtauP, jalphaP, jband2;
    // resting rigid boxes (Sec. 4.2.1); face_ok bit 2a+s: face (axis a,
    // side s) is not on the domain boundary
    int n_obst;
    // obstacle boxes and the cell size in binary64 in both precisions: which
    // nodes lie in a box and which face is nearest are decided as the
    // reference decides them, not by binary32 rounding of positions that sit
    // on a face
    double obst_lo[kMaxObstacles][3], obst_hi[kMaxObstacles][3], obst_h;
    int obst_face_ok[kMaxObstacles];
};

// One buffer of particle state, component-major with stride cap.
//   x[D], v[D], C[D*D], then SAND, ELASTIC: G[D*D] (= F_e - I), S[D(D+1)/2]
//                            FLUID: dJ[1] (= J - 1), S[1]
//                            VFLUID, JAUMANN: dJ[1], S[D(D+1)/2]
template <class T>
struct PView {
    T* x;
    T* v;
    T* C;
    T* G;      // F_e - I, or dJ = J - 1
    T* S;
    int32_t* pid;
    long long cap;
};

struct ActiveTile {
    int tile, off, cnt, pad;
};

}  // namespace mpm
