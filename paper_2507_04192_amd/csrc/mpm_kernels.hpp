// Forward MPM step kernels for gfx950 and their host launchers.
//
// One step (Sec. 2.2, update-stress-last):
//   1. scan_reduce / scan_down  tile histogram -> tile offsets, active tiles
//   2. bucket                   particles scattered into their tile's range
//   3. p2g                      one tile per workgroup: cell-level stable sort
//                               in LDS, then P2G (eq:update_m, momentum with the
//                               APIC affine term of App. B, internal force from
//                               the stress cache) into the tile's LDS node
//                               block, written out as the tile's partial block
//   4. grid                     sums the partial blocks covering each node in
//                               a fixed order; v = P/m + dt g, walls (Sec. 5.3
//                               friction law).  No floating-point atomics: the
//                               step is deterministic.
//   5. g2p                      per active tile: LDS node block, velocity,
//                               APIC C, velocity gradient, position, then the
//                               constitutive update; writes the state in the
//                               new sorted order and counts the next keys
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "mpm_device.hpp"
#include "mpm_runtime.hpp"

namespace mpm {

template <int D> struct TileShape;
template <> struct TileShape<3> { static constexpr int TE = 4, BE = 6, NB = 216; };
template <> struct TileShape<2> { static constexpr int TE = 8, BE = 10, NB = 100; };

constexpr int kSortCap = 1024;   // particles per tile sorted in LDS (larger: in perm)
// threads of a P2G workgroup, one tile each: binary64 one wave; binary32 two
// waves that share the tile's particles and split the node values between
// them (mass and momentum x | the other momentum components)
// With FLIP the node values double (momentum with and without the internal
// force): binary32 then uses four waves per tile.
template <class T, bool FL = false> constexpr int kP2GBlock = sizeof(T) == 4 ? (FL ? 256 : 128) : 64;
template <class T, bool FL = false> constexpr int kP2GWGs = kTileWGs * kBlock / kP2GBlock<T, FL>;
// threads of a G2P workgroup (binary64: smaller groups, measured faster)
template <class T> constexpr int kG2PBlock = sizeof(T) == 8 ? 128 : 256;
// G2P loads the next tile's node block while it works on the current one
// (binary64: measured faster; binary32: slower)
template <class T> constexpr bool kG2PPrefetch = sizeof(T) == 8;
constexpr int kGridBlock = 128;  // threads of a grid-update workgroup

// Particle data read once per step (P2G's inputs, G2P's old state) and the
// part of G2P's output that no later kernel of the step reads (F or J, pid)
// go through the non-temporal cache hint.  Measured on the 3-D cylinder:
// binary32 P2G 106 -> 98 us, G2P 140 -> 137 us, binary64 P2G 200 -> 192,
// G2P 256 -> 246; the hint on the stores that P2G reads next (x, v, C, the
// stress cache) made G2P slower, so those stay ordinary stores.
template <class T>
__device__ __forceinline__ T ld_once(const T* p)
{
    return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void st_late(T v, T* p)
{
    __builtin_nontemporal_store(v, p);
}

// Active-list entry handled by this workgroup on iteration `it`.  Workgroup b
// runs on XCD b % 8; each XCD gets one contiguous chunk of the active list so
// that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int tile_entry(int it, int n_active)
{
    int nx = 8;
    int per = gridDim.x / nx;
    int xcd = blockIdx.x % nx;
    int lb = blockIdx.x / nx;
    int chunk = (n_active + nx - 1) / nx;
    int e = xcd * chunk + lb + it * per;
    int end = min((xcd + 1) * chunk, n_active);
    return e < end ? e : -1;
}

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of two ints (256 threads).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void block_scan2(int a, int b, int& ex_a, int& ex_b, int& tot_a, int& tot_b)
{
    __shared__ int sa[4], sb[4];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int ia = a, ib = b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int ta = __shfl_up(ia, o), tb = __shfl_up(ib, o);
        if (lane >= o) { ia += ta; ib += tb; }
    }
    if (lane == 63) { sa[w] = ia; sb[w] = ib; }
    __syncthreads();
    int pa = 0, pb = 0;
    for (int k = 0; k < w; ++k) { pa += sa[k]; pb += sb[k]; }
    tot_a = sa[0] + sa[1] + sa[2] + sa[3];
    tot_b = sb[0] + sb[1] + sb[2] + sb[3];
    ex_a = pa + ia - a;
    ex_b = pb + ib - b;
    __syncthreads();
}

template <int Unused = 0>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int* __restrict__ count, int ntiles,
                                                        int* __restrict__ part)
{
    int base = blockIdx.x * kScanChunk;
    int s = 0, a = 0;
    for (int i = threadIdx.x; i < kScanChunk; i += kBlock) {
        int t = base + i;
        if (t < ntiles) {
            int c = count[t];
            s += c;
            a += (c > 0);
        }
    }
    int es, ea, ts, ta;
    block_scan2(s, a, es, ea, ts, ta);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ts;
        part[2 * blockIdx.x + 1] = ta;
    }
}

template <int Unused = 0>
__global__ __launch_bounds__(kBlock) void k_scan_down(const int* __restrict__ count, int ntiles,
                                                      const int* __restrict__ part,
                                                      int* __restrict__ tile_off, int* __restrict__ tile_slot,
                                                      ActiveTile* __restrict__ active, int* __restrict__ meta)
{
    // prefix of the earlier chunks
    int ps = 0, pa = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += kBlock) {
        ps += part[2 * i];
        pa += part[2 * i + 1];
    }
    int e0, e1, base_s, base_a;
    block_scan2(ps, pa, e0, e1, base_s, base_a);
    constexpr int PER = kScanChunk / kBlock;
    int t0 = blockIdx.x * kScanChunk + threadIdx.x * PER;
    int c[PER];
    int ls = 0, la = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int t = t0 + k;
        c[k] = (t < ntiles) ? count[t] : 0;
        ls += c[k];
        la += (c[k] > 0);
    }
    int ex_s, ex_a, tot_s, tot_a;
    block_scan2(ls, la, ex_s, ex_a, tot_s, tot_a);
    int off = base_s + ex_s, slot = base_a + ex_a;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int t = t0 + k;
        if (t < ntiles) {
            tile_off[t] = off;
            if (c[k] > 0) {
                tile_slot[t] = slot;
                ActiveTile e;
                e.tile = t;
                e.off = off;
                e.cnt = c[k];
                e.pad = 0;
                active[slot] = e;
                ++slot;
            } else {
                tile_slot[t] = -1;
            }
        }
        off += c[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) {
        meta[0] = slot;
        meta[1] = off;
    }
}

// Scatter every particle into its tile's range (order inside a tile is
// arbitrary here; the P2G kernel sorts it).  Leaves count[] at zero.  A
// thread takes kBucketPer particles, kBlock apart, whose loads, range
// reservations and stores are each issued together.
constexpr int kBucketPer = 4;

template <int Unused = 0>
__global__ __launch_bounds__(kBlock) void k_bucket(long long N, const int* __restrict__ key,
                                                   int* __restrict__ count, const int* __restrict__ tile_off,
                                                   int* __restrict__ tmp, int* __restrict__ tmpk)
{
    const long long j0 = (long long)blockIdx.x * (kBlock * kBucketPer) + threadIdx.x;
    int k[kBucketPer], head[kBucketPer], len[kBucketPer], rank[kBucketPer], base[kBucketPer];
#pragma unroll
    for (int q = 0; q < kBucketPer; ++q) {
        const long long j = j0 + q * kBlock;
        k[q] = j < N ? key[j] : -1;
    }
#pragma unroll
    for (int q = 0; q < kBucketPer; ++q) {
        const bool valid = j0 + q * kBlock < N;
        wave_runs(valid ? (k[q] >> 6) : -1, valid, head[q], len[q], rank[q]);
        base[q] = 0;
        if (valid && rank[q] == 0) base[q] = atomicSub(&count[k[q] >> 6], len[q]) - len[q];
    }
#pragma unroll
    for (int q = 0; q < kBucketPer; ++q) {
        const long long j = j0 + q * kBlock;
        const int b = __shfl(base[q], head[q]);
        if (j < N) {
            const int slot = tile_off[k[q] >> 6] + b + rank[q];
            tmp[slot] = (int)j;
            tmpk[slot] = k[q];
        }
    }
}

template <class T, int D>
__global__ __launch_bounds__(kBlock) void k_keys(Geo g, Phys<T> P, PView<T> cur, long long N,
                                                 int* __restrict__ key, int* __restrict__ count)
{
    long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
    bool valid = j < N;
    int k = 0;
    if (valid) {
        T xp[D];
#pragma unroll
        for (int a = 0; a < D; ++a) xp[a] = cur.x[a * cur.cap + j];
        k = cell_key<T, D>(g, xp, P.inv);
        key[j] = k;
    }
    int head, len, rank;
    wave_runs(valid ? (k >> 6) : -1, valid, head, len, rank);
    if (valid && rank == 0) atomicAdd(&count[k >> 6], len);
}

// ---------------------------------------------------------------------------
// P2G
// ---------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ void weights_from_f(T f, T inv, T w[3], T dw[3])
{
    T a0 = T(1.5) - f, a1 = f - T(1), a2 = f - T(0.5);
    w[0] = T(0.5) * a0 * a0;
    w[1] = T(0.75) - a1 * a1;
    w[2] = T(0.5) * a2 * a2;
    dw[0] = -a0 * inv;
    dw[1] = T(-2) * a1 * inv;
    dw[2] = a2 * inv;
}

// Orders this wave's LDS accesses: the compiler may not move LDS reads or
// writes across it, and the hardware executes one wave's LDS operations in
// order, so a lane sees what another lane of the same wave wrote before.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The state of one particle that P2G reads for the momentum components
// [A0, A1): the position, those components of v, those rows of C and the
// stress cache.
template <class T, int D, int MAT, int A0 = 0, int A1 = D>
struct P2GIn {
    static constexpr int NS = mat_iso_stress(MAT) ? 1 : D * (D + 1) / 2;
    static constexpr int NA = A1 - A0;
    T x[D], v[NA], C[NA * D], S[NS];
    __device__ __forceinline__ void load(const PView<T>& cur, int j)
    {
        const long long cap = cur.cap;
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = ld_once(&cur.x[a * cap + j]);
#pragma unroll
        for (int a = 0; a < NA; ++a) v[a] = ld_once(&cur.v[(A0 + a) * cap + j]);
#pragma unroll
        for (int q = 0; q < NA * D; ++q) C[q] = ld_once(&cur.C[(A0 * D + q) * cap + j]);
#pragma unroll
        for (int q = 0; q < NS; ++q) S[q] = ld_once(&cur.S[q * cap + j]);
    }
};

// Index of entry (a, b) in the packed symmetric storage of the stress cache
// (3-D: 00 11 22 01 02 12; 2-D: 00 11 01).
template <int D>
__host__ __device__ constexpr int sym_index(int a, int b)
{
    return a == b ? a : (D == 2 ? 2 : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5)));
}

// One particle's P2G contribution (eq:update_m, the momentum with the APIC
// affine term of App. B, and the internal force -dt V_p sigma_p grad phi).
// Every weight factors over the axes, so per node line along x the terms
// that do not depend on x are formed once.  With wyz = w_y w_z (2-D: w_y),
// the values at node (kx, line) are
//   mass  w_x mw,                              mw  = m_p wyz,
//   P_a   w_x U_a + (w_x dd_x) V_a + dw_x W_a,
//   U_a = wyz (m v_a + sum_{b>0} mC_ab dd_b) + sum_{b>0} fs_ab (grad phi_b / w_x),
//   V_a = wyz mC_a0,  W_a = wyz fs_a0.
// For each of the 3^D stencil nodes, sink(k, n, fx, mw, U, V, W, Uq)
// receives the offset index k, the node's index n in the tile's LDS block,
// the x factors fx = (w_x, w_x dd_x, dw_x) and the line terms of the
// momentum components [A0, A1); Uq = wyz (m v_a + ...) is U without the
// force, so the momentum without the internal force is w_x Uq + (w_x dd_x) V
// (FLIP's v_i^n); p2g_node_values forms the D+1 values from them when the
// range is all of them.
template <class T, int D, int MAT, int A0, int A1, class Sink>
__device__ __forceinline__ void p2g_particle(const Phys<T>& P, const P2GIn<T, D, MAT, A0, A1>& in, const int lb[3],
                                             const int gb[3], Sink&& sink)
{
    constexpr int BE = TileShape<D>::BE, NA = A1 - A0;
    T w[D][3], dw[D][3], dd[D][3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T x = in.x[a];
        T t = mul_exact(x, P.inv);
        T f = t - T(gb[a]);
        weights_from_f(f, P.inv, w[a], dw[a]);
#pragma unroll
        for (int k = 0; k < 3; ++k) dd[a][k] = (T(k) - f) * P.h;
    }
    // rows A0..A1-1 of m v, m C and fs = -dt V sigma
    T mv[NA], mC[NA][D], fs[NA][D];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        mv[a] = P.mass * in.v[a];
#pragma unroll
        for (int b = 0; b < D; ++b) {
            mC[a][b] = P.mass * in.C[a * D + b];
            if constexpr (mat_iso_stress(MAT)) fs[a][b] = (A0 + a == b) ? -P.dt * in.S[0] : T(0);
            else fs[a][b] = -P.dt * in.S[sym_index<D>(A0 + a, b)];
        }
    }
    T fx[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        fx[q][0] = w[0][q];
        fx[q][1] = w[0][q] * dd[0][q];
        fx[q][2] = dw[0][q];
    }
    constexpr int KZ = (D == 3) ? 3 : 1;
#pragma unroll
    for (int kz = 0; kz < KZ; ++kz) {
        T mvz[NA];   // m v_a + mC_a2 dd_z: the part of the affine term fixed on a z plane
#pragma unroll
        for (int a = 0; a < NA; ++a) mvz[a] = (D == 3) ? mv[a] + mC[a][D - 1] * dd[D - 1][kz] : mv[a];
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            T wyz = (D == 3) ? w[1][ky] * w[2][kz] : w[1][ky];
            T g1 = (D == 3) ? dw[1][ky] * w[2][kz] : dw[1][ky];
            T g2 = (D == 3) ? w[1][ky] * dw[2][kz] : T(0);
            T U[NA], V[NA], Wf[NA], Uq[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                T aff = mvz[a] + mC[a][1] * dd[1][ky];
                Uq[a] = wyz * aff;
                T u = Uq[a] + fs[a][1] * g1;
                if constexpr (D == 3) u += fs[a][2] * g2;
                U[a] = u;
                V[a] = wyz * mC[a][0];
                Wf[a] = wyz * fs[a][0];
            }
            T mw = P.mass * wyz;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                int n;
                if constexpr (D == 3) n = ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] + kx;
                else n = (lb[1] + ky) * BE + lb[0] + kx;
                sink((kz * 3 + ky) * 3 + kx, n, fx[kx], mw, U, V, Wf, Uq);
            }
        }
    }
}

// The D+1 values (mass, momentum) a particle adds at one node, from the
// factors p2g_particle hands to its sink.
template <class T, int D>
__device__ __forceinline__ void p2g_node_values(const T fx[3], T mw, const T U[D], const T V[D], const T W[D],
                                                T add[D + 1])
{
    add[0] = fx[0] * mw;
#pragma unroll
    for (int a = 0; a < D; ++a) add[1 + a] = fx[0] * U[a] + fx[1] * V[a] + fx[2] * W[a];
}

// Node index in the tile's LDS block of stencil offset k for a lane whose
// cell sits at lb.
template <int D>
__device__ __forceinline__ int block_node(const int lb[3], int k)
{
    constexpr int BE = TileShape<D>::BE;
    int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
    if constexpr (D == 3) return ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] + kx;
    else return (lb[1] + ky) * BE + lb[0] + kx;
}

// Position inside its tile of the particle of rank q in cell c, for the
// order (rank, cell): all cells' rank-0 particles first, then rank 1, ...
//   pos = sum_c' min(cnt[c'], q) + #{c' < c : cnt[c'] > q}.
// For q < 64 the two sums come from a table (the cells with more than q
// particles as a 64-bit mask, and the running count of earlier ranks);
// deeper ranks, which only crowded cells reach, count directly.
__device__ __forceinline__ int rank_major_pos(int c, int q, const unsigned long long* rmask, const int* roff,
                                              const int* cnt)
{
    if (q < 64) return roff[q] + __popcll(rmask[q] & ((1ull << c) - 1ull));
    // read through volatile: keeps the compiler from hoisting the 64 counts
    // into registers out of the callers' particle loops
    const volatile int* vc = cnt;
    int r = 0;
#pragma unroll 1
    for (int c2 = 0; c2 < 64; ++c2) {
        int n = vc[c2];
        r += min(n, q) + ((c2 < c && n > q) ? 1 : 0);
    }
    return r;
}

// Binary32 P2G of one lane (cell) for the momentum components [A0, A1)
// (and the mass when MASS): the lane sums the particles of its cell in
// registers (they all hit the same 3^D nodes), the next particle's state
// loaded while this one is spread, then adds its sums to node arrays
// [Q0, Q0 + NQ) of the tile's LDS block.  With QV the sums are those of the
// momentum without the internal force (node arrays 1 + D + a, for FLIP).
// The lanes of a wave write distinct nodes per offset and wave_sync orders
// the offsets.
template <class T, int D, int MAT, int A0, int A1, bool MASS, bool QV>
__device__ __forceinline__ void p2g_lane_sums(const Phys<T>& P, const PView<T>& cur, const int* sorted, int lane,
                                              int mycnt, const int lb[3], const int gb[3],
                                              const unsigned long long* s_rmask, const int* s_roff,
                                              const int* s_cnt, T (*node)[TileShape<D>::NB])
{
    static_assert(!(MASS && QV), "the mass travels with the momentum including the force");
    constexpr int NK = (D == 3) ? 27 : 9;
    constexpr int M = MASS ? 1 : 0;
    constexpr int NQ = M + A1 - A0;             // node values of this wave
    constexpr int Q0 = M ? 0 : (QV ? 1 + D + A0 : 1 + A0);   // its first node array
    T acc[NK][NQ];
#pragma unroll
    for (int k = 0; k < NK; ++k)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[k][q] = T(0);
    P2GIn<T, D, MAT, A0, A1> nx;
    if (mycnt > 0) nx.load(cur, sorted[rank_major_pos(lane, 0, s_rmask, s_roff, s_cnt)]);
    for (int r = 0; r < mycnt; ++r) {
        const P2GIn<T, D, MAT, A0, A1> in = nx;
        if (r + 1 < mycnt) nx.load(cur, sorted[rank_major_pos(lane, r + 1, s_rmask, s_roff, s_cnt)]);
        // the products go straight into the sums (one FMA each)
        p2g_particle<T, D, MAT, A0, A1>(P, in, lb, gb,
                                        [&](int k, int, const T* fx, T mw, const T* U, const T* V, const T* W,
                                            const T* Uq) {
            if constexpr (MASS) acc[k][0] = fma(fx[0], mw, acc[k][0]);
#pragma unroll
            for (int a = 0; a < A1 - A0; ++a) {
                if constexpr (QV) acc[k][M + a] = fma(fx[1], V[a], fma(fx[0], Uq[a], acc[k][M + a]));
                else acc[k][M + a] = fma(fx[2], W[a], fma(fx[1], V[a], fma(fx[0], U[a], acc[k][M + a])));
            }
        });
    }
    if (mycnt > 0) {
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            int n = block_node<D>(lb, k);
            T cv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) cv[q] = node[Q0 + q][n];
#pragma unroll
            for (int q = 0; q < NQ; ++q) node[Q0 + q][n] = cv[q] + acc[k][q];
            wave_sync();
        }
    } else {
#pragma unroll
        for (int k = 0; k < NK; ++k) wave_sync();
    }
}

// P2G, one tile per workgroup.  The workgroup (1) sorts the tile's particles
// into perm: by rank within their cell (previous slot order), then by cell,
// so that the r-th particles of the 64 cells are adjacent in memory; (2)
// takes them in rounds, lane c holding the r-th particle of cell c for
// r = 0, 1, ... (the lanes of a round read adjacent slots), binary32 with
// two waves that split the node values; (3) writes the tile's node block
// (mass, momentum; with FLIP also the momentum without the internal force)
// to its partial block.  Register budget: three waves per SIMD in binary32
// (168 registers), two in binary64.
template <class T, int D, int MAT, bool FL>
__global__ __launch_bounds__((kP2GBlock<T, FL>)) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2))) void k_p2g(Geo g, Phys<T> P, const int* __restrict__ meta,
                                                const ActiveTile* __restrict__ active, int* __restrict__ tmp,
                                                const int* __restrict__ tmpk, PView<T> cur, int* __restrict__ perm,
                                                T* __restrict__ part)
{
    constexpr int TE = TileShape<D>::TE, NB = TileShape<D>::NB;
    constexpr int NT = kP2GBlock<T, FL>;
    constexpr int NV = FL ? 2 * D + 1 : D + 1;          // node values per block node
    constexpr bool kRegAcc = sizeof(T) == 4;            // binary32: sums in registers
    __shared__ T s_node[NV][NB];
    __shared__ int s_cnt[64], s_off[64], s_cur[64];
    __shared__ int s_unord[kSortCap], s_sorted[kSortCap];
    __shared__ unsigned char s_ucell[kSortCap];
    __shared__ int s_max;
    __shared__ unsigned long long s_rmask[64];
    __shared__ int s_roff[64];
    const int n_active = meta[0];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int it = 0;; ++it) {
        int e = tile_entry(it, n_active);
        if (e < 0) break;
        const ActiveTile at = active[e];
        for (int i = tid; i < NV * NB; i += NT) (&s_node[0][0])[i] = T(0);
        if (tid < 64) { s_cnt[tid] = 0; s_cur[tid] = 0; }
        __syncthreads();
        const bool in_lds = at.cnt <= kSortCap;
        // A tile that fits in LDS keeps its particles' cells and slots in
        // registers (thread t holds entries t, t + NT, ...): one batch of global
        // loads instead of one round trip per pass below.
        constexpr int KPL = (kSortCap + NT - 1) / NT;   // register slots per thread: KPL * NT >= kSortCap
        static_assert(KPL * NT >= kSortCap, "the register batch must cover an in-LDS tile");
        const int nk = at.cnt - tid;                 // entry i * NT of this thread exists if below
        const int* tk = tmpk + at.off + tid;
        const int* tj = tmp + at.off + tid;
        int rc[KPL], rj[KPL];
        if (in_lds) {
#pragma unroll
            for (int i = 0; i < KPL; ++i)
                if (i * NT < nk) {
                    rc[i] = tk[i * NT] & 63;   // the cell is the low 6 bits of the key
                    rj[i] = tj[i * NT];
                }
#pragma unroll
            for (int i = 0; i < KPL; ++i)
                if (i * NT < nk) atomicAdd(&s_cnt[rc[i]], 1);
        } else {
            for (int k = tid; k < at.cnt; k += NT) atomicAdd(&s_cnt[tmpk[at.off + k] & 63], 1);
        }
        __syncthreads();
        if (tid < 64) {
            int v = s_cnt[lane], inc = v, mx = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                int t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
                mx = max(mx, __shfl_xor(mx, o));
            }
            s_off[lane] = inc - v;
            if (lane == 0) s_max = mx;
            // rank table: cells with more than q particles, earlier ranks' count
            int run = 0;
            const int lim = mx < 64 ? mx : 64;
            for (int q = 0; q < lim; ++q) {
                unsigned long long m = __ballot(v > q);
                if (lane == 0) {
                    s_rmask[q] = m;
                    s_roff[q] = run;
                }
                run += __popcll(m);
            }
        }
        __syncthreads();
        if (in_lds) {
            // place each particle in its cell's range (arbitrary order inside)
            // and note the cell of each position; then rank every particle
            // inside its cell by previous slot: a stable order
#pragma unroll
            for (int i = 0; i < KPL; ++i) {
                if (i * NT >= nk) continue;
                const int u = s_off[rc[i]] + atomicAdd(&s_cur[rc[i]], 1);
                s_unord[u] = rj[i];
                s_ucell[u] = (unsigned char)rc[i];
            }
            __syncthreads();
            for (int u = tid; u < at.cnt; u += NT) {
                const int c = s_ucell[u], j = s_unord[u];
                const int o = s_off[c], n = s_cnt[c], last = o + n - 1;
                int rank = 0;
                // four independent LDS reads per pass; reads past the cell's
                // range repeat its last entry and are not counted
                for (int q = 0; q < n; q += 4) {
                    int e[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) e[i] = s_unord[min(o + q + i, last)];
#pragma unroll
                    for (int i = 0; i < 4; ++i) rank += (q + i < n && e[i] < j) ? 1 : 0;
                }
                s_sorted[rank_major_pos(c, rank, s_rmask, s_roff, s_cnt)] = j;
            }
            __syncthreads();
            for (int k = tid; k < at.cnt; k += NT) perm[at.off + k] = s_sorted[k];
        } else {
            // crowded tile: the same placement and rank-by-counting, with the
            // cell-major placement in perm and the rank-major result staged in
            // this tile's range of tmp (its bucketed input is no longer
            // needed), then copied back to perm
            int* unord = perm + at.off;
            for (int k = tid; k < at.cnt; k += NT) {
                int c = tmpk[at.off + k] & 63;
                int pos = atomicAdd(&s_cur[c], 1);
                unord[s_off[c] + pos] = tmp[at.off + k];
            }
            __threadfence_block();
            __syncthreads();
            for (int k = tid; k < at.cnt; k += NT) {
                int p = k, lo = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1)
                    if (lo + step < 64 && s_off[lo + step] <= p) lo += step;
                const int j = unord[p], o = s_off[lo], n = s_cnt[lo];
                int rank = 0;
                for (int q = 0; q < n; ++q) rank += unord[o + q] < j;
                tmp[at.off + rank_major_pos(lo, rank, s_rmask, s_roff, s_cnt)] = j;
            }
            __threadfence_block();
            __syncthreads();
            const volatile int* rm = tmp + at.off;
            for (int k = tid; k < at.cnt; k += NT) unord[k] = rm[k];
            __threadfence_block();
            __syncthreads();
        }
        const int* sorted = in_lds ? s_sorted : (perm + at.off);
        int tc[3];
        tile_coords(g, at.tile, tc);
        // The lane's cell, made opaque to the compiler for this tile: what is
        // derived from it (node offsets, LDS addresses) is then formed per
        // tile instead of being hoisted out of the tile loop, where it would
        // hold registers through the particle loop.
        int cl = lane;
        asm volatile("" : "+v"(cl));
        int lb[3], gb[3];
        lb[0] = cl % TE;
        lb[1] = (cl / TE) % TE;
        lb[2] = (D == 3) ? cl / (TE * TE) : 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) gb[a] = tc[a] * TE + lb[a] - g.G;
        const int mycnt = s_cnt[cl], maxc = s_max;
        if constexpr (kRegAcc) {
            // binary32: lane c of each wave sums the particles of cell c in
            // registers (they all hit the same 3^D nodes), wave 0 the mass and
            // momentum x, wave 1 the other momentum components, then adds its
            // sums to the tile's LDS block; the waves write different node
            // arrays, the lanes of a wave distinct nodes per offset, and
            // wave_sync orders the offsets
            // (with FLIP, waves 2 and 3 the same for the momentum without the
            // internal force)
            T (*node)[NB] = s_node;
            if (w == 0)
                p2g_lane_sums<T, D, MAT, 0, 1, true, false>(P, cur, sorted, cl, mycnt, lb, gb, s_rmask, s_roff, s_cnt, node);
            else if (w == 1)
                p2g_lane_sums<T, D, MAT, 1, D, false, false>(P, cur, sorted, cl, mycnt, lb, gb, s_rmask, s_roff, s_cnt, node);
            else if constexpr (FL) {
                if (w == 2)
                    p2g_lane_sums<T, D, MAT, 0, 1, false, true>(P, cur, sorted, cl, mycnt, lb, gb, s_rmask, s_roff, s_cnt, node);
                else
                    p2g_lane_sums<T, D, MAT, 1, D, false, true>(P, cur, sorted, cl, mycnt, lb, gb, s_rmask, s_roff, s_cnt, node);
            }
        } else {
            // binary64 (one wave): hardware LDS atomics (ds_add_f64) into the
            // tile's block, issued without waiting; lanes hit distinct nodes
            // per offset, so the summation order is fixed
            for (int r = 0; r < maxc; ++r) {
                if (r < mycnt) {
                    P2GIn<T, D, MAT> in;
                    in.load(cur, sorted[rank_major_pos(cl, r, s_rmask, s_roff, s_cnt)]);
                    p2g_particle<T, D, MAT>(P, in, lb, gb,
                                            [&](int, int n, const T* fx, T mw, const T* U, const T* V, const T* W,
                                                const T* Uq) {
                        T add[D + 1];
                        p2g_node_values<T, D>(fx, mw, U, V, W, add);
#pragma unroll
                        for (int q = 0; q <= D; ++q) atomicAdd(&s_node[q][n], add[q]);
                        if constexpr (FL)
#pragma unroll
                            for (int a = 0; a < D; ++a) atomicAdd(&s_node[1 + D + a][n], fma(fx[1], V[a], fx[0] * Uq[a]));
                    });
                }
            }
        }
        __syncthreads();
        T* dst = part + (long long)e * NV * NB;
        for (int i = tid; i < NV * NB; i += NT) dst[i] = (&s_node[0][0])[i];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Grid update over the node blocks of the active tiles.  A node shared by
// several blocks is handled by exactly one of them: the first active tile
// among its candidates, own tile first.  Its mass and momentum are the sum of
// the partial blocks that cover it, in that same fixed order.
// ---------------------------------------------------------------------------

// The partial blocks that cover block node I (global node coordinates):
// candidate msk takes its own tile minus one along every axis whose bit is
// set, own tile first.  Writes each candidate's active slot (-1: none) and
// the node's index in that block, and returns the node's owner tile: the
// first active candidate (-1 if none).  All slots are loaded before any is
// used.
template <int D>
__device__ __forceinline__ int node_blocks(const Geo& g, const int I[3], const int own[3], const bool down[3],
                                           const int* __restrict__ tile_slot, int slot[1 << D], int li[1 << D])
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NC = 1 << D;
    int tl[NC];
#pragma unroll
    for (int msk = 0; msk < NC; ++msk) {
        bool ok = true;
        int ct[3] = {own[0], own[1], own[2]};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if ((msk >> a) & 1) {
                if (!down[a]) ok = false;
                ct[a] -= 1;
            }
            if (ct[a] >= g.ntile[a]) ok = false;
        }
        tl[msk] = (ct[2] * g.ntile[1] + ct[1]) * g.ntile[0] + ct[0];
        if constexpr (D == 3) li[msk] = ((I[2] - ct[2] * TE) * BE + I[1] - ct[1] * TE) * BE + I[0] - ct[0] * TE;
        else li[msk] = (I[1] - ct[1] * TE) * BE + I[0] - ct[0] * TE;
        slot[msk] = ok ? tile_slot[tl[msk]] : -1;
    }
    int des = -1;
#pragma unroll
    for (int msk = NC - 1; msk >= 0; --msk)
        if (slot[msk] >= 0) des = tl[msk];
    return des;
}

// With FL (FLIP) the partial blocks also hold the momentum without the
// internal force, and gvo receives the velocity before the update,
// v_i^n = that / m_i (0 where m_i = 0).  Resting obstacles (Sec. 4.2.1) act
// after the walls.
template <class T, int D, bool FL>
__global__ __launch_bounds__(kGridBlock) void k_grid(Geo g, Phys<T> P, const int* __restrict__ meta,
                                                 const ActiveTile* __restrict__ active,
                                                 const int* __restrict__ tile_slot, const T* __restrict__ part,
                                                 T* __restrict__ gv, T* __restrict__ gmass, T* __restrict__ gvt,
                                                 T* __restrict__ gvo)
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NB = TileShape<D>::NB;
    constexpr int NV = FL ? 2 * D + 1 : D + 1;
    const int n_active = meta[0];
    for (int it = 0;; ++it) {
        int e = tile_entry(it, n_active);
        if (e < 0) break;
        int tile = active[e].tile;
        int tc[3];
        tile_coords(g, tile, tc);
        for (int i = threadIdx.x; i < NB; i += kGridBlock) {
            int l[3] = {i % BE, (i / BE) % BE, (D == 3) ? i / (BE * BE) : 0};
            int I[3], own[3];
            bool down[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                I[a] = (a < D) ? tc[a] * TE + l[a] : 0;
                own[a] = I[a] / TE;
                down[a] = (a < D) && (I[a] % TE < 2) && own[a] >= 1;
            }
            constexpr int NC = 1 << D;
            int slot[NC], li[NC];
            const int des = node_blocks<D>(g, I, own, down, tile_slot, slot, li);
            T m = T(0), p[D], pq[FL ? D : 1];
#pragma unroll
            for (int a = 0; a < D; ++a) p[a] = T(0);
            if constexpr (FL)
#pragma unroll
                for (int a = 0; a < D; ++a) pq[a] = T(0);
            if (des == tile) {
#pragma unroll
                for (int msk = 0; msk < NC; ++msk) {
                    if (slot[msk] < 0) continue;
                    const T* src = part + (long long)slot[msk] * NV * NB;
                    m += src[li[msk]];
#pragma unroll
                    for (int a = 0; a < D; ++a) p[a] += src[(1 + a) * NB + li[msk]];
                    if constexpr (FL)
#pragma unroll
                        for (int a = 0; a < D; ++a) pq[a] += src[(1 + D + a) * NB + li[msk]];
                }
            }
            if (des != tile) continue;
            long long node = node_index(g, I[0], I[1], I[2]);
            T v[D];
#pragma unroll
            for (int a = 0; a < D; ++a) v[a] = T(0);
            if (m > T(0)) {
#pragma unroll
                for (int a = 0; a < D; ++a) v[a] = p[a] / m + P.dt * P.g[a];
                if (gvt)
#pragma unroll
                    for (int a = 0; a < D; ++a) gvt[a * g.NN + node] = v[a];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    int ip = I[a] - g.G;
                    if (ip <= 0) {
                        T mu = P.wall_mu[2 * a];
                        if (a == D - 1 && P.floor_mu) {
                            int fx = min(I[0], g.box[0] - 1);
                            int fi = (D == 3) ? min(I[1], g.box[1] - 1) * P.floor_stride + fx : fx;
                            mu = P.floor_mu[fi];
                        }
                        wall_node<T, D>(P.wall_mode[2 * a], mu, a, T(-1), v);
                    }
                    if (ip >= g.n[a]) wall_node<T, D>(P.wall_mode[2 * a + 1], P.wall_mu[2 * a + 1], a, T(1), v);
                }
                if (P.n_obst > 0) {
                    double xi[D];
#pragma unroll
                    for (int a = 0; a < D; ++a) xi[a] = double(I[a] - g.G) * P.obst_h;
                    obstacle_node<T, D>(P, xi, v);
                }
            } else if (gvt) {
#pragma unroll
                for (int a = 0; a < D; ++a) gvt[a * g.NN + node] = T(0);
            }
#pragma unroll
            for (int a = 0; a < D; ++a) gv[a * g.NN + node] = v[a];
            if constexpr (FL)
#pragma unroll
                for (int a = 0; a < D; ++a) gvo[a * g.NN + node] = m > T(0) ? pq[a] / m : T(0);
            if (P.keep_grid) gmass[node] = m;
        }
    }
}

// ---------------------------------------------------------------------------
// G2P + kinematics + constitutive
// ---------------------------------------------------------------------------

// Nodal velocities of a tile's LDS block (the tile's nodes and its halo), NPT
// block nodes per thread: thread t takes nodes t, t + NT, ...
template <class T, int D, int NPT, int NT>
__device__ __forceinline__ void g2p_block_load(const Geo& g, const T* __restrict__ gv, int tile, int tid,
                                               T r[D][NPT])
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NB = TileShape<D>::NB;
    int tc[3];
    tile_coords(g, tile, tc);
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        const int i = tid + p * NT;
        if (i < NB) {
            int l0 = i % BE, l1 = (i / BE) % BE, l2 = (D == 3) ? i / (BE * BE) : 0;
            long long node = node_index(g, tc[0] * TE + l0, tc[1] * TE + l1, (D == 3) ? tc[2] * TE + l2 : 0);
#pragma unroll
            for (int a = 0; a < D; ++a) r[a][p] = gv[a * g.NN + node];
        }
    }
}

// The transfer (App. B) sets the new velocity and the carried matrix C:
// APIC C = (4/h^2) sum phi v_i (x_i - x_p)^T, TPIC C = the velocity gradient,
// PIC and FLIP C = 0; FLIP (FL) also gathers the grid velocity before the
// update, gvo, and blends: v' = sum phi v_i + alpha (v_p - sum phi v_i^n).
template <class T, int D, int MAT, int XF>
__global__ __launch_bounds__(kG2PBlock<T>) void k_g2p(Geo g, Phys<T> P, const int* __restrict__ meta,
                                                const ActiveTile* __restrict__ active, const int* __restrict__ perm,
                                                PView<T> cur, PView<T> nxt, const T* __restrict__ gv,
                                                const T* __restrict__ gvo,
                                                int* __restrict__ key_out, int* __restrict__ count,
                                                int* __restrict__ status, const T* __restrict__ eps_in,
                                                T* __restrict__ eps_out)
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NB = TileShape<D>::NB;
    constexpr int NS = D * (D + 1) / 2;
    constexpr int NPT = (NB + kG2PBlock<T> - 1) / kG2PBlock<T>;   // block nodes per thread
    constexpr bool FL = XF == XF_FLIP;
    __shared__ T s_v[D][NB];
    __shared__ T s_vo[FL ? D : 1][FL ? NB : 1];
    const int n_active = meta[0];
    const int tid = threadIdx.x;
    const long long cap = cur.cap;
    // With kG2PPrefetch, the next tile's node velocities are loaded into
    // registers while this tile's particles are processed (and its
    // active-list entry one tile earlier still); otherwise each tile loads its
    // own block at its top.
    constexpr bool PF = kG2PPrefetch<T> && !FL;
    int e = __builtin_amdgcn_readfirstlane(tile_entry(0, n_active));
    if (e < 0) return;
    ActiveTile at = active[e];
    T pre[D][NPT];
    if (PF) g2p_block_load<T, D, NPT, kG2PBlock<T>>(g, gv, at.tile, tid, pre);
    int en = __builtin_amdgcn_readfirstlane(tile_entry(1, n_active));
    int next_tile = (PF && en >= 0) ? active[en].tile : 0;
    for (int it = 0; e >= 0; ++it) {
        if (!PF) g2p_block_load<T, D, NPT, kG2PBlock<T>>(g, gv, at.tile, tid, pre);
        if constexpr (FL) {
            T preo[D][NPT];
            g2p_block_load<T, D, NPT, kG2PBlock<T>>(g, gvo, at.tile, tid, preo);
#pragma unroll
            for (int p = 0; p < NPT; ++p) {
                const int i = tid + p * kG2PBlock<T>;
                if (i < NB)
#pragma unroll
                    for (int a = 0; a < D; ++a) s_vo[a][i] = preo[a][p];
            }
        }
#pragma unroll
        for (int p = 0; p < NPT; ++p) {
            const int i = tid + p * kG2PBlock<T>;
            if (i < NB)
#pragma unroll
                for (int a = 0; a < D; ++a) s_v[a][i] = pre[a][p];
        }
        __syncthreads();
        int enn = -1, next2_tile = 0;
        if (!PF) {
            enn = __builtin_amdgcn_readfirstlane(tile_entry(it + 2, n_active));
        } else if (en >= 0) {
            g2p_block_load<T, D, NPT, kG2PBlock<T>>(g, gv, next_tile, tid, pre);
            enn = __builtin_amdgcn_readfirstlane(tile_entry(it + 2, n_active));
            if (enn >= 0) next2_tile = active[enn].tile;
        }
        int tc[3];
        tile_coords(g, at.tile, tc);
        for (int k0 = 0; k0 < at.cnt; k0 += kG2PBlock<T>) {
            int k = k0 + tid;
            bool valid = k < at.cnt;
            int newkey = 0;
            if (valid) {
                long long s = at.off + k;
                int j = ld_once(&perm[s]);
                T xp[D], w[D][3], dw[D][3], dd[D][3];
                int lb[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    xp[a] = ld_once(&cur.x[a * cap + j]);
                    int b;
                    T f;
                    stencil_axis(xp[a], P.inv, b, f, w[a], dw[a]);
                    int l = b + g.G - tc[a] * TE;
                    lb[a] = l < 0 ? 0 : (l > TE - 1 ? TE - 1 : l);   // memory guard only
#pragma unroll
                    for (int q = 0; q < 3; ++q) dd[a][q] = (T(q) - f) * P.h;
                }
                // Gather over the 3^D stencil nodes of the LDS block:
                //   vn = sum phi v,  Bm = sum phi v (x_i - x_p)^T,  Lm = sum v (grad phi)^T.
                // Each weight is a product of per-axis factors: every node
                // line along x is reduced with the x factors (w, w dd, dw),
                // then combined with the line's y/z factors.  The scheduling
                // barrier after each line keeps the compiler from hoisting
                // all LDS reads of the stencil (registers, occupancy).
                T vn[D], Bm[D][D], Lm[D][D], vo[FL ? D : 1];
                {
                    constexpr int NL = (D == 3) ? 9 : 3;
                    T wdx[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) wdx[q] = w[0][q] * dd[0][q];
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        vn[a] = T(0);
                        if constexpr (FL) vo[a] = T(0);
#pragma unroll
                        for (int b = 0; b < D; ++b) { Bm[a][b] = T(0); Lm[a][b] = T(0); }
                    }
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        const int ky = l % 3, kz = l / 3;
                        const T lw = (D == 3) ? w[1][ky] * w[2][kz] : w[1][ky];
                        const T ld1 = lw * dd[1][ky];
                        const T ldw1 = (D == 3) ? dw[1][ky] * w[2][kz] : dw[1][ky];
                        const int n0 = (D == 3) ? ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] : (lb[1] + ky) * BE + lb[0];
#pragma unroll
                        for (int a = 0; a < D; ++a) {
                            T v0 = s_v[a][n0], v1 = s_v[a][n0 + 1], v2 = s_v[a][n0 + 2];
                            T A0 = w[0][0] * v0 + w[0][1] * v1 + w[0][2] * v2;
                            T A1 = wdx[0] * v0 + wdx[1] * v1 + wdx[2] * v2;
                            T A2 = dw[0][0] * v0 + dw[0][1] * v1 + dw[0][2] * v2;
                            vn[a] += lw * A0;
                            Bm[a][0] += lw * A1;
                            Bm[a][1] += ld1 * A0;
                            Lm[a][0] += lw * A2;
                            Lm[a][1] += ldw1 * A0;
                            if constexpr (D == 3) {
                                Bm[a][2] += (lw * dd[2][kz]) * A0;
                                Lm[a][2] += (w[1][ky] * dw[2][kz]) * A0;
                            }
                            if constexpr (FL)
                                vo[a] += lw * (w[0][0] * s_vo[a][n0] + w[0][1] * s_vo[a][n0 + 1] +
                                               w[0][2] * s_vo[a][n0 + 2]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                bool bad = false, fast = false, noconv = false;
                T xn[D];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    T xv = xp[a] + P.dt * vn[a];
                    bad |= !finite(xv) || !finite(vn[a]);
                    fast |= fabs(P.dt * vn[a]) > P.h;   // moved more than a cell: CFL violated
                    xv = fmin(fmax(xv, T(0)), P.ext[a]);
                    xn[a] = xv;
                    nxt.x[a * cap + s] = xv;
                    if constexpr (FL) {
                        const T vf = vn[a] + P.flip_alpha * (cur.v[a * cap + j] - vo[a]);
                        bad |= !finite(vf);
                        nxt.v[a * cap + s] = vf;
#pragma unroll
                        for (int b = 0; b < D; ++b) nxt.C[(a * D + b) * cap + s] = T(0);
                    } else {
                        nxt.v[a * cap + s] = vn[a];
#pragma unroll
                        for (int b = 0; b < D; ++b) {
                            T cab;
                            if constexpr (XF == XF_APIC) cab = P.Dinv * Bm[a][b];
                            else if constexpr (XF == XF_TPIC) cab = Lm[a][b];
                            else cab = T(0);
                            nxt.C[(a * D + b) * cap + s] = cab;
                        }
                    }
                }
                if constexpr (MAT == MAT_FLUID) {
                    T dJ = ld_once(&cur.G[j]), si;
                    fluid_update<T, D>(P, Lm, dJ, si);
                    bad |= !finite(si) || !finite(dJ);
                    st_late(dJ, &nxt.G[s]);
                    nxt.S[s] = si;
                } else if constexpr (MAT == MAT_VFLUID || MAT == MAT_JAUMANN) {
                    T dJ = ld_once(&cur.G[j]), Sv[NS];
                    if constexpr (MAT == MAT_JAUMANN)   // the viscous fluid's stress is a function of J and L
#pragma unroll
                        for (int q = 0; q < NS; ++q) Sv[q] = cur.S[q * cap + j];
                    if constexpr (MAT == MAT_VFLUID) vfluid_update<T, D>(P, Lm, dJ, Sv);
                    else {
                        // equivalent plastic strain (when carried): App. A's increment
                        T de;
                        jaumann_update<T, D>(P, Lm, dJ, Sv, &de);
                        if (eps_out) eps_out[s] = ld_once(&eps_in[j]) + de;
                    }
                    bad |= !finite(dJ);
                    st_late(dJ, &nxt.G[s]);
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        bad |= !finite(Sv[q]);
                        nxt.S[q * cap + s] = Sv[q];
                    }
                } else {
                    T Gm[D][D], Sv[NS];
#pragma unroll
                    for (int a = 0; a < D; ++a)
#pragma unroll
                        for (int b = 0; b < D; ++b) Gm[a][b] = ld_once(&cur.G[(a * D + b) * cap + j]);
                    T dgam;
                    noconv = !hencky_update<T, D>(P, MAT == MAT_SAND, Lm, Gm, Sv, &dgam);
                    // equivalent plastic strain (when carried): sqrt(2/3) |dE_p|
                    if (MAT == MAT_SAND && eps_out) eps_out[s] = ld_once(&eps_in[j]) + T(0.816496580927726) * dgam;
#pragma unroll
                    for (int a = 0; a < D; ++a)
#pragma unroll
                        for (int b = 0; b < D; ++b) st_late(Gm[a][b], &nxt.G[(a * D + b) * cap + s]);
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        bad |= !finite(Sv[q]);
                        nxt.S[q * cap + s] = Sv[q];
                    }
                }
                int pid = ld_once(&cur.pid[j]);
                st_late(pid, &nxt.pid[s]);
                if (bad) {
                    atomicOr(&status[0], 1);
                    atomicMin(&status[1], pid);
                }
                if (fast) {
                    atomicOr(&status[0], 2);
                    atomicMin(&status[2], pid);
                }
                if (noconv) {
                    atomicOr(&status[0], 4);
                    atomicMin(&status[3], pid);
                }
                newkey = cell_key<T, D>(g, xn, P.inv);
                key_out[s] = newkey;
            }
            int head, len, rank;
            wave_runs(valid ? (newkey >> 6) : -1, valid, head, len, rank);
            if (valid && rank == 0) atomicAdd(&count[newkey >> 6], len);
        }
        __syncthreads();
        e = en;
        if (e >= 0) at = active[e];
        en = enn;
        next_tile = next2_tile;
    }
}

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------

template <class T>
__global__ void k_fill(T* p, long long n, T v)
{
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    long long stride = (long long)gridDim.x * kBlock;
    for (; i < n; i += stride) p[i] = v;
}

// Particle field copy between the ABI layout (ncomp x N, memory or pid order)
// and the workspace layout (ncomp x cap, memory order), with the stored-form
// conversions: F = I + G, J = 1 + dJ, symmetric S <-> full dim x dim.
enum { CONV_COPY = 0, CONV_ADD_IDENTITY = 1, CONV_ADD_ONE = 2, CONV_SYM = 3, CONV_ISO = 4 };

template <class T, int D>
__global__ void k_read_field(const T* __restrict__ src, long long cap, const int32_t* __restrict__ pid,
                             long long N, int ncomp, int conv, int by_pid, T* __restrict__ dst)
{
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    long long o = by_pid ? pid[s] : s;
    for (int c = 0; c < ncomp; ++c) {
        T v;
        int a = c / D, b = c % D;
        switch (conv) {
        case CONV_ADD_IDENTITY: v = src[c * cap + s] + ((a == b) ? T(1) : T(0)); break;
        case CONV_ADD_ONE: v = src[s] + T(1); break;
        case CONV_SYM: {
            int q;
            if (D == 3) q = (a == b) ? a : ((a + b == 1) ? 3 : ((a + b == 2) ? 4 : 5));
            else q = (a == b) ? a : 2;
            v = src[q * cap + s];
            break;
        }
        case CONV_ISO: v = (a == b) ? src[s] : T(0); break;
        default: v = src[c * cap + s];
        }
        dst[c * N + o] = v;
    }
}

template <class T, int D>
__global__ void k_write_field(T* __restrict__ dst, long long cap, const int32_t* __restrict__ pid,
                              long long N, int ncomp, int conv, int by_pid, const T* __restrict__ src)
{
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    long long o = by_pid ? pid[s] : s;
    if (conv == CONV_SYM) {
        if (D == 3) {
            dst[0 * cap + s] = src[0 * N + o];
            dst[1 * cap + s] = src[4 * N + o];
            dst[2 * cap + s] = src[8 * N + o];
            dst[3 * cap + s] = T(0.5) * (src[1 * N + o] + src[3 * N + o]);
            dst[4 * cap + s] = T(0.5) * (src[2 * N + o] + src[6 * N + o]);
            dst[5 * cap + s] = T(0.5) * (src[5 * N + o] + src[7 * N + o]);
        } else {
            dst[0 * cap + s] = src[0 * N + o];
            dst[1 * cap + s] = src[3 * N + o];
            dst[2 * cap + s] = T(0.5) * (src[1 * N + o] + src[2 * N + o]);
        }
        return;
    }
    if (conv == CONV_ISO) {
        T tr = T(0);
        for (int a = 0; a < D; ++a) tr += src[(a * D + a) * N + o];
        dst[s] = tr / T(D);
        return;
    }
    for (int c = 0; c < ncomp; ++c) {
        int a = c / D, b = c % D;
        T v = src[c * N + o];
        if (conv == CONV_ADD_IDENTITY) v -= (a == b) ? T(1) : T(0);
        if (conv == CONV_ADD_ONE) v -= T(1);
        dst[c * cap + s] = v;
    }
}

template <int Unused = 0>
__global__ void k_iota(int32_t* p, long long n)
{
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

// Dense node box (n + 1 + 2G per axis) from the tile-padded grid.  The grid
// kernel writes only the node blocks of the step's active tiles, so a node
// that no active tile's block covers holds a value of an earlier step; it is
// read as zero (no mass, no velocity), which is what the step's grid holds
// there.  tile_slot[t] >= 0 marks the active tiles of the step.
template <class T>
__global__ void k_read_grid(Geo g, const T* __restrict__ src, int ncomp, const int* __restrict__ tile_slot,
                            T* __restrict__ dst)
{
    long long nbox = (long long)g.box[0] * g.box[1] * g.box[2];
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nbox) return;
    int I[3];
    I[0] = (int)(i % g.box[0]);
    long long r = i / g.box[0];
    I[1] = (int)(r % g.box[1]);
    I[2] = (int)(r / g.box[1]);
    // tiles whose (T+2)-node block holds the node: own = I / T, and own - 1
    // where I lies in the first two nodes of its tile
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        int own = (a < g.dim) ? I[a] / g.T : 0;
        hi[a] = own;
        lo[a] = (a < g.dim && I[a] % g.T < 2 && own >= 1) ? own - 1 : own;
    }
    bool live = false;
    for (int tz = lo[2]; tz <= hi[2]; ++tz)
        for (int ty = lo[1]; ty <= hi[1]; ++ty)
            for (int tx = lo[0]; tx <= hi[0]; ++tx)
                live |= tile_slot[((long long)tz * g.ntile[1] + ty) * g.ntile[0] + tx] >= 0;
    long long node = node_index(g, I[0], I[1], I[2]);
    for (int c = 0; c < ncomp; ++c) dst[c * nbox + i] = live ? src[c * g.NN + node] : T(0);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

inline unsigned nblocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <class T>
Phys<T> make_phys(const mpm_ctx* c, double dt)
{
    Phys<T> P{};
    const mpm_config& k = c->cfg;
    int D = k.dim;
    P.h = (T)k.dx;
    P.inv = T(1) / (T)k.dx;
    P.Dinv = T(4) / ((T)k.dx * (T)k.dx);
    P.dt = (T)dt;
    P.mass = (T)c->mass;
    P.vol0 = (T)c->vol0;
    for (int a = 0; a < 3; ++a) {
        P.g[a] = (T)k.gravity[a];
        P.ext[a] = (a < D) ? (T)((double)k.n[a] * k.dx) : T(0);
    }
    double E = k.youngs, nu = k.poisson;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    double s = sin(k.phi_deg * M_PI / 180.0);
    double q_phi = 6.0 * s / (sqrt(3.0) * (3.0 + s));
    double alpha = sqrt(2.0) / 3.0 * q_phi;
    P.lam = (T)lam;
    P.mu = (T)mu;
    P.cone_coef = (T)((D * lam + 2.0 * mu) / (2.0 * mu) * alpha);
    P.k_over_gamma = (T)(k.bulk / k.gamma);
    P.gamma = (T)k.gamma;
    P.material = c->mat;
    for (int f = 0; f < 6; ++f) {
        P.wall_mode[f] = k.wall_mode[f];
        P.wall_mu[f] = (T)k.wall_mu[f];
    }
    P.floor_mu = (const T*)c->floor_mu;
    P.floor_stride = c->geo.box[0];
    P.keep_grid = k.keep_grid;
    P.xfer = c->xfer;
    P.flip_alpha = (T)k.flip_alpha;
    P.visc = (T)k.viscosity;
    {
        // hypoelastic Drucker-Prager constants (App. A)
        double sp = sin(k.phi_deg * M_PI / 180.0), cp = cos(k.phi_deg * M_PI / 180.0);
        double ss = sin(k.psi_deg * M_PI / 180.0);
        double q_phi = 6.0 * sp / (sqrt(3.0) * (3.0 + sp));
        double k_phi = 6.0 * k.cohesion * cp / (sqrt(3.0) * (3.0 + sp));
        double q_psi = 6.0 * ss / (sqrt(3.0) * (3.0 + ss));
        P.jK = (T)(lam + 2.0 * mu / D);
        P.jq_phi = (T)q_phi;
        P.jk_phi = (T)k_phi;
        P.jq_psi = (T)q_psi;
        P.jst = (T)k.tension;
        P.jtauP = (T)(k_phi - q_phi * k.tension);
        P.jalphaP = (T)(sqrt(1.0 + q_phi * q_phi) - q_phi);
        P.jband2 = (T)(1e-6 * E * 1e-6 * E);
    }
    P.n_obst = k.n_obstacles;
    P.obst_h = k.dx;
    for (int o = 0; o < kMaxObstacles; ++o) {
        int ok = 0;
        for (int a = 0; a < 3; ++a) {
            P.obst_lo[o][a] = k.obst_lo[o][a];
            P.obst_hi[o][a] = k.obst_hi[o][a];
            if (a < D) {
                double ext = (double)k.n[a] * k.dx;
                if (k.obst_lo[o][a] > 0.0) ok |= 1 << (2 * a);        // lower face inside the domain
                if (k.obst_hi[o][a] < ext) ok |= 1 << (2 * a + 1);    // upper face inside the domain
            }
        }
        P.obst_face_ok[o] = ok;
    }
    return P;
}

template <class T>
PView<T> view(const mpm_ctx* c, int which)
{
    PView<T> v{};
    T* base = (T*)c->st[which];
    long long cap = c->cap;
    int D = c->cfg.dim;
    v.cap = cap;
    v.x = base;
    v.v = base + D * cap;
    v.C = base + 2 * D * cap;
    v.G = base + (2 * D + D * D) * cap;
    v.S = v.G + (mat_has_F(c->mat) ? D * D : 1) * cap;
    v.pid = c->pid[which];
    return v;
}

template <class T, int D>
struct Solver {
    static int launch_err(mpm_ctx* c, const char* what) { return hip_check(c, hipGetLastError(), what); }

    static int init_particles(mpm_ctx* c, const void* x, const void* v)
    {
        PView<T> s = view<T>(c, c->cur);
        long long N = c->N, cap = c->cap;
        hipStream_t st = c->stream;
        for (int a = 0; a < D; ++a) {
            if (hipMemcpyAsync(s.x + a * cap, (const T*)x + a * N, sizeof(T) * N, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(s.v + a * cap, (const T*)v + a * N, sizeof(T) * N, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return launch_err(c, "init copy");
        }
        // C, G (or dJ) and S start at zero: they follow v contiguously
        long long rest = (long long)(c->nsc - 2 * D) * cap;
        if (rest > 0) k_fill<T><<<std::min<long long>(nblocks(rest), 4096), kBlock, 0, st>>>(s.C, rest, T(0));
        if (N > 0) k_iota<0><<<nblocks(N), kBlock, 0, st>>>(s.pid, N);
        for (int i = 0; i < 2; ++i)
            if (c->eps[i]) k_fill<T><<<std::min<long long>(nblocks(cap), 4096), kBlock, 0, st>>>((T*)c->eps[i], cap, T(0));
        return recompute_keys(c);
    }

    static int recompute_keys(mpm_ctx* c)
    {
        hipStream_t st = c->stream;
        k_fill<int><<<std::min<long long>(nblocks(c->geo.ntiles), 4096), kBlock, 0, st>>>(c->count, c->geo.ntiles, 0);
        if (c->N > 0) {
            Phys<T> P = make_phys<T>(c, 0.0);
            k_keys<T, D><<<nblocks(c->N), kBlock, 0, st>>>(c->geo, P, view<T>(c, c->cur), c->N, c->key, c->count);
        }
        return launch_err(c, "keys");
    }

    static int clear_grid(mpm_ctx* c)
    {
        hipStream_t st = c->stream;
        long long NN = c->geo.NN;
        k_fill<T><<<4096, kBlock, 0, st>>>((T*)c->gv, D * NN, T(0));
        k_fill<T><<<4096, kBlock, 0, st>>>((T*)c->gmass, NN, T(0));
        if (c->gvo) k_fill<T><<<4096, kBlock, 0, st>>>((T*)c->gvo, D * NN, T(0));
        k_fill<int><<<1, kBlock, 0, st>>>(c->status, 16, 0);
        k_fill<int><<<1, kBlock, 0, st>>>(c->status + 1, 3, 0x7fffffff);
        if (c->geo.ntiles > 0)
            k_fill<int><<<std::min<long long>(nblocks(c->geo.ntiles), 4096), kBlock, 0, st>>>(c->tile_slot, c->geo.ntiles, -1);
        return launch_err(c, "clear grid");
    }

    // Where one step keeps its sort and grid: the context's own arrays, or a
    // record of the grid tape (then the nodal velocity before the walls is
    // kept too, for the adjoint).
    struct StepBufs {
        int32_t* perm;
        int32_t* tile_slot;
        ActiveTile* active;
        int32_t* meta;
        T* gv;
        T* gmass;
        T* gvt;
        T* gvo;     // FLIP: nodal velocity before the update
        const T* eps_in = nullptr;   // equivalent plastic strain, when carried
        T* eps_out = nullptr;
    };
    static StepBufs ctx_bufs(mpm_ctx* c)
    {
        return {c->perm, c->tile_slot, c->active, c->meta, (T*)c->gv, (T*)c->gmass, nullptr, (T*)c->gvo};
    }

    // One step from state view cur into state view nxt with the transfer XF
    // (FLIP: P2G and the grid update also form the velocity before the
    // update).  The transfer is a template parameter: as a run-time choice it
    // kept both affine candidates live in G2P and cost it half its waves.
    template <int MAT, int XF = XF_APIC>
    static void step_views(mpm_ctx* c, const Phys<T>& P, const PView<T>& cur, const PView<T>& nxt,
                           const StepBufs& b)
    {
        constexpr bool FL = XF == XF_FLIP;
        // P2G depends on the material only through the stored stress: one
        // isotropic value or the symmetric tensor
        constexpr int PM = mat_iso_stress(MAT) ? MAT_FLUID : MAT_SAND;
        hipStream_t st = c->stream;
        const Geo& g = c->geo;
        unsigned nsb = (unsigned)((g.ntiles + kScanChunk - 1) / kScanChunk);
        prof_mark(c, -1);
        // one chunk has no earlier chunks to sum: the down-sweep alone (a
        // launch fewer for the small grids, whose steps are launch-bound)
        if (nsb > 1) k_scan_reduce<0><<<nsb, kBlock, 0, st>>>(c->count, g.ntiles, c->part);
        k_scan_down<0><<<nsb, kBlock, 0, st>>>(c->count, g.ntiles, c->part, c->tile_off, b.tile_slot, b.active, b.meta);
        prof_mark(c, MPM_PROF_SCAN);
        k_bucket<0><<<(unsigned)((c->N + kBlock * kBucketPer - 1) / (kBlock * kBucketPer)), kBlock, 0, st>>>(
            c->N, c->key, c->count, c->tile_off, c->tmp, c->tmpk);
        prof_mark(c, MPM_PROF_BUCKET);
        k_p2g<T, D, PM, FL><<<kP2GWGs<T, FL>, kP2GBlock<T, FL>, 0, st>>>(g, P, b.meta, b.active, c->tmp, c->tmpk, cur,
                                                                        b.perm, (T*)c->part_grid);
        prof_mark(c, MPM_PROF_P2G);
        k_grid<T, D, FL><<<kTileWGs * kBlock / kGridBlock, kGridBlock, 0, st>>>(g, P, b.meta, b.active, b.tile_slot, (const T*)c->part_grid,
                                                  b.gv, b.gmass, b.gvt, b.gvo);
        prof_mark(c, MPM_PROF_GRID);
        k_g2p<T, D, MAT, XF><<<kTileWGs * kBlock / kG2PBlock<T>, kG2PBlock<T>, 0, st>>>(g, P, b.meta, b.active, b.perm, cur, nxt, (const T*)b.gv,
                                                      (const T*)b.gvo, c->key, c->count, c->status, b.eps_in, b.eps_out);
        prof_mark(c, MPM_PROF_G2P);
    }

    template <int MAT, int XF = XF_APIC>
    static void step_views(mpm_ctx* c, const Phys<T>& P, const PView<T>& cur, const PView<T>& nxt)
    {
        step_views<MAT, XF>(c, P, cur, nxt, ctx_bufs(c));
    }

    template <int MAT, int XF>
    static void one_step(mpm_ctx* c, const Phys<T>& P)
    {
        StepBufs b = ctx_bufs(c);
        if ((MAT == MAT_SAND || MAT == MAT_JAUMANN) && c->eps[0]) {
            b.eps_in = (const T*)c->eps[c->cur];
            b.eps_out = (T*)c->eps[1 - c->cur];
        }
        step_views<MAT, XF>(c, P, view<T>(c, c->cur), view<T>(c, 1 - c->cur), b);
        c->cur = 1 - c->cur;
    }

    template <int XF>
    static void one_step_x(mpm_ctx* c, const Phys<T>& P)
    {
        switch (c->mat) {
        case MAT_FLUID: one_step<MAT_FLUID, XF>(c, P); break;
        case MAT_SAND: one_step<MAT_SAND, XF>(c, P); break;
        case MAT_VFLUID: one_step<MAT_VFLUID, XF>(c, P); break;
        case MAT_JAUMANN: one_step<MAT_JAUMANN, XF>(c, P); break;
        default: one_step<MAT_ELASTIC, XF>(c, P); break;
        }
    }

    static int step(mpm_ctx* c, int n, double dt)
    {
        Phys<T> P = make_phys<T>(c, dt);
        for (int i = 0; i < n; ++i) {
            switch (c->xfer) {
            case XF_PIC: one_step_x<XF_PIC>(c, P); break;
            case XF_FLIP: one_step_x<XF_FLIP>(c, P); break;
            case XF_TPIC: one_step_x<XF_TPIC>(c, P); break;
            default: one_step_x<XF_APIC>(c, P); break;
            }
        }
        return launch_err(c, "step");
    }

    // field -> (pointer into state, ncomp in ABI layout, conversion)
    static int field_desc(mpm_ctx* c, int field, T** ptr, int* ncomp, int* conv)
    {
        PView<T> s = view<T>(c, c->cur);
        const bool fluid = !mat_has_F(c->mat);   // carries J instead of F
        const bool iso = mat_iso_stress(c->mat);
        switch (field) {
        case MPM_FIELD_X: *ptr = s.x; *ncomp = D; *conv = CONV_COPY; return MPM_OK;
        case MPM_FIELD_V: *ptr = s.v; *ncomp = D; *conv = CONV_COPY; return MPM_OK;
        case MPM_FIELD_C: *ptr = s.C; *ncomp = D * D; *conv = CONV_COPY; return MPM_OK;
        case MPM_FIELD_F:
            if (fluid) break;
            *ptr = s.G; *ncomp = D * D; *conv = CONV_ADD_IDENTITY; return MPM_OK;
        case MPM_FIELD_FMI:
            if (fluid) break;
            *ptr = s.G; *ncomp = D * D; *conv = CONV_COPY; return MPM_OK;
        case MPM_FIELD_J:
            if (!fluid) break;
            *ptr = s.G; *ncomp = 1; *conv = CONV_ADD_ONE; return MPM_OK;
        case MPM_FIELD_JM1:
            if (!fluid) break;
            *ptr = s.G; *ncomp = 1; *conv = CONV_COPY; return MPM_OK;
        case MPM_FIELD_STRESS:
            *ptr = s.S; *ncomp = D * D; *conv = iso ? CONV_ISO : CONV_SYM; return MPM_OK;
        case MPM_FIELD_EPS_EQ:
            if (!c->eps[c->cur]) return set_err(c, MPM_EINVAL, "EPS_EQ needs track_eps_eq = 1");
            *ptr = (T*)c->eps[c->cur]; *ncomp = 1; *conv = CONV_COPY; return MPM_OK;
        default: break;
        }
        return set_err(c, MPM_EINVAL, "field not available for this material");
    }

    static int read_state(mpm_ctx* c, int field, int order, void* dst)
    {
        hipStream_t st = c->stream;
        PView<T> s = view<T>(c, c->cur);
        long long N = c->N;
        if (field == MPM_FIELD_PID) {
            if (order == MPM_ORDER_PID) return set_err(c, MPM_EINVAL, "pid in pid order is the identity");
            if (hipMemcpyAsync(dst, s.pid, sizeof(int32_t) * N, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return launch_err(c, "read pid");
            return MPM_OK;
        }
        T* src;
        int ncomp, conv;
        int rc = field_desc(c, field, &src, &ncomp, &conv);
        if (rc) return rc;
        if (N > 0)
            k_read_field<T, D><<<nblocks(N), kBlock, 0, st>>>(src, c->cap, s.pid, N, ncomp, conv,
                                                             order == MPM_ORDER_PID, (T*)dst);
        return launch_err(c, "read state");
    }

    static int write_state(mpm_ctx* c, int field, int order, const void* src)
    {
        hipStream_t st = c->stream;
        PView<T> s = view<T>(c, c->cur);
        long long N = c->N;
        if (field == MPM_FIELD_PID) return set_err(c, MPM_EINVAL, "pid cannot be written");
        T* dstp;
        int ncomp, conv;
        int rc = field_desc(c, field, &dstp, &ncomp, &conv);
        if (rc) return rc;
        if (N > 0)
            k_write_field<T, D><<<nblocks(N), kBlock, 0, st>>>(dstp, c->cap, s.pid, N, ncomp, conv,
                                                              order == MPM_ORDER_PID, (const T*)src);
        rc = launch_err(c, "write state");
        if (rc) return rc;
        if (field == MPM_FIELD_X) return recompute_keys(c);
        return MPM_OK;
    }

    static int read_grid(mpm_ctx* c, int which, void* dst)
    {
        const Geo& g = c->geo;
        long long nbox = (long long)g.box[0] * g.box[1] * g.box[2];
        if (which == MPM_GRID_MASS) {
            if (!c->cfg.keep_grid) return set_err(c, MPM_EINVAL, "grid mass needs keep_grid = 1");
            k_read_grid<T><<<nblocks(nbox), kBlock, 0, c->stream>>>(g, (const T*)c->gmass, 1, c->tile_slot, (T*)dst);
        } else if (which == MPM_GRID_VEL) {
            k_read_grid<T><<<nblocks(nbox), kBlock, 0, c->stream>>>(g, (const T*)c->gv, D, c->tile_slot, (T*)dst);
        } else {
            return set_err(c, MPM_EINVAL, "unknown grid field");
        }
        return launch_err(c, "read grid");
    }

    static Ops table()
    {
        Ops o;
        o.init_particles = &init_particles;
        o.recompute_keys = &recompute_keys;
        o.clear_grid = &clear_grid;
        o.step = &step;
        o.read_state = &read_state;
        o.write_state = &write_state;
        o.read_grid = &read_grid;
        return o;
    }
};

}  // namespace mpm
