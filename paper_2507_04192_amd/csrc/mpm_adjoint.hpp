// Adjoint of the MPM step for gfx950 and the checkpointed rollout driver.
//
// Forward (mpm_forward_loss): the state is copied to a checkpoint every k
// steps; at observation frames the extraction operators Q_l and the masked
// squared error are evaluated on the device (loss in binary64).
//
// Backward (mpm_backward), segment by segment from the last: the segment's
// checkpoint is restored and its k steps recomputed into a tape of states
// and a grid tape (each step's sort, nodal mass and nodal velocity before
// and after the walls); then for each step in reverse (Sec. 3.1, eq:dzda;
// Sec. 3.3 recomputation):
//   g2p_adj   per particle: reverse of the constitutive update and of G2P;
//             node adjoints accumulated in LDS and written per tile
//   grid_adj  per node: reverse of the walls (dL/dmu) and of v = P/m + dt g
//   p2g_adj   per particle: reverse of P2G, then the sort is undone by
//             writing each particle's adjoint at its slot before the step.
#pragma once

#include "mpm_adjoint_device.hpp"
#include "mpm_kernels.hpp"

namespace mpm {

constexpr int kAdjBlock = 128;   // threads of the reverse per-tile kernels

// Per-slot intermediate of the reverse sweep (mid), component-major with
// stride cap, written by k_g2p_adj and read by k_p2g_adj:
//   [0, D)              position adjoint
//   [D, D + D^2)        adjoint of the stored F_e - I (fluid: [D] holds J;
//                       hypoelastic Drucker-Prager: [D] J, then the
//                       constitutive part of the packed stress adjoint in
//                       [D + 1, D + 1 + D(D+1)/2), which fits the same slots)
//   [D + D^2, 2D + D^2) FLIP: the direct adjoint of the input velocity,
//                       alpha times that of v'
template <int D> struct MidLayout {
    static constexpr int X = 0, G = D, S = D + 1, V = D + D * D, N = D + D * D;
    static_assert(D + 1 + D * (D + 1) / 2 <= D + D * D, "stress adjoint fits the intermediate");
};

// Reverse of the constitutive update, the kinematics x' = x + dt v and G2P,
// per particle of a tile.  First part: recomputes the G2P velocity and
// velocity gradient from the tile's node block and applies the constitutive
// VJP.  Second part, line by line: node adjoints of the velocity
// (accumulated in binary64 in LDS, then written as the tile's partial block)
// and the position adjoint through the weights and x_i - x_p.  The velocity,
// velocity-gradient and partial position adjoints pass between the parts in
// registers; the F (or J) adjoint and the position adjoint go to mid.
// FLIP (FL): v' = sum phi v_i + alpha (v_p - sum phi v_i^n); the adjoint of
// v^n = sum phi v_i^n is scattered to a second node block (binary64 LDS,
// written after the first in the tile's partial block), its weights pass
// an adjoint to the position, and alpha times the adjoint of v' goes to mid
// as the direct adjoint of v_p.
template <class T, int D, int MAT, bool FL>
__global__ __launch_bounds__(kAdjBlock) void k_g2p_adj(Geo g, Phys<T> P, const int* __restrict__ meta,
                                                    const ActiveTile* __restrict__ active,
                                                    const int* __restrict__ perm, PView<T> st, PView<T> aout,
                                                    const T* __restrict__ gv, const T* __restrict__ gvo,
                                                    T* __restrict__ part, T* __restrict__ mid)
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NB = TileShape<D>::NB;
    constexpr int NS = D * (D + 1) / 2;
    constexpr int NVA = FL ? 2 * D + 1 : D + 1;   // partial block values per node
    using ML = MidLayout<D>;
    __shared__ T s_v[D][NB];
    __shared__ double s_b[D][NB];
    __shared__ T s_vo[FL ? D : 1][FL ? NB : 1];
    __shared__ double s_bo[FL ? D : 1][FL ? NB : 1];
    const int n_active = meta[0];
    const int tid = threadIdx.x;
    const long long cap = st.cap;
    const T inv2 = P.inv * P.inv;
    for (int it = 0;; ++it) {
        int e = tile_entry(it, n_active);
        if (e < 0) break;
        ActiveTile at = active[e];
        int tc[3];
        tile_coords(g, at.tile, tc);
        for (int i = tid; i < NB; i += kAdjBlock) {
            int l0 = i % BE, l1 = (i / BE) % BE, l2 = (D == 3) ? i / (BE * BE) : 0;
            long long node = node_index(g, tc[0] * TE + l0, tc[1] * TE + l1, (D == 3) ? tc[2] * TE + l2 : 0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                s_v[a][i] = gv[a * g.NN + node];
                s_b[a][i] = 0.0;
                if constexpr (FL) {
                    s_vo[a][i] = gvo[a * g.NN + node];
                    s_bo[a][i] = 0.0;
                }
            }
        }
        __syncthreads();
        for (int k = tid; k < at.cnt; k += kAdjBlock) {
            long long s = at.off + k;
            int j = perm[s];
            T xbar_c[D], vt_c[D], Lb_c[D][D], vob_c[FL ? D : 1];
            {
                T xp[D], w[D][3], dw[D][3];
                int lb[3] = {0, 0, 0};
    #pragma unroll
                for (int a = 0; a < D; ++a) {
                    xp[a] = st.x[a * cap + j];
                    int b;
                    T f;
                    stencil_axis(xp[a], P.inv, b, f, w[a], dw[a]);
                    int l = b + g.G - tc[a] * TE;
                    lb[a] = l < 0 ? 0 : (l > TE - 1 ? TE - 1 : l);
                }
                // forward G2P of this particle: velocity and velocity gradient,
                // line by line along x as in the forward kernel (per-axis weight
                // factors; a scheduling barrier per line bounds register use)
                T vn[D], Lm[D][D];
                {
                    constexpr int NL = (D == 3) ? 9 : 3;
    #pragma unroll
                    for (int a = 0; a < D; ++a) {
                        vn[a] = T(0);
    #pragma unroll
                        for (int b = 0; b < D; ++b) Lm[a][b] = T(0);
                    }
    #pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        const int ky = l % 3, kz = l / 3;
                        const T lw = (D == 3) ? w[1][ky] * w[2][kz] : w[1][ky];
                        const T ldw1 = (D == 3) ? dw[1][ky] * w[2][kz] : dw[1][ky];
                        const int n0 = (D == 3) ? ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] : (lb[1] + ky) * BE + lb[0];
    #pragma unroll
                        for (int a = 0; a < D; ++a) {
                            T v0 = s_v[a][n0], v1 = s_v[a][n0 + 1], v2 = s_v[a][n0 + 2];
                            T A0 = w[0][0] * v0 + w[0][1] * v1 + w[0][2] * v2;
                            T A2 = dw[0][0] * v0 + dw[0][1] * v1 + dw[0][2] * v2;
                            vn[a] += lw * A0;
                            Lm[a][0] += lw * A2;
                            Lm[a][1] += ldw1 * A0;
                            if constexpr (D == 3) Lm[a][2] += (w[1][ky] * dw[2][kz]) * A0;
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                // reverse of the constitutive update
                T Lb[D][D];
                if constexpr (MAT == MAT_FLUID) {
                    T Jb_in;
                    fluid_vjp<T, D>(P, Lm, st.G[j], aout.G[s], aout.S[s], Lb, Jb_in);
                    mid[ML::G * cap + s] = Jb_in;
                } else if constexpr (MAT == MAT_VFLUID) {
                    T sb[NS], Jb_in;
    #pragma unroll
                    for (int q = 0; q < NS; ++q) sb[q] = aout.S[q * cap + s];
                    vfluid_vjp<T, D>(P, Lm, st.G[j], aout.G[s], sb, Lb, Jb_in);
                    mid[ML::G * cap + s] = Jb_in;
                } else if constexpr (MAT == MAT_JAUMANN) {
                    T Sv[NS], sb[NS], sb_in[NS], Jb_in;
    #pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        Sv[q] = st.S[q * cap + j];
                        sb[q] = aout.S[q * cap + s];
                    }
                    jaumann_vjp<T, D>(P, Lm, st.G[j], Sv, aout.G[s], sb, Lb, Jb_in, sb_in);
                    mid[ML::G * cap + s] = Jb_in;
    #pragma unroll
                    for (int q = 0; q < NS; ++q) mid[(ML::S + q) * cap + s] = sb_in[q];
                } else {
                    T G[D][D], Gb[D][D], Gb_in[D][D], sb[NS];
    #pragma unroll
                    for (int a = 0; a < D; ++a)
    #pragma unroll
                        for (int b = 0; b < D; ++b) {
                            G[a][b] = st.G[(a * D + b) * cap + j];
                            Gb[a][b] = aout.G[(a * D + b) * cap + s];
                        }
    #pragma unroll
                    for (int q = 0; q < NS; ++q) sb[q] = aout.S[q * cap + s];
                    hencky_vjp<T, D>(P, MAT == MAT_SAND, Lm, G, Gb, sb, Lb, Gb_in);
    #pragma unroll
                    for (int a = 0; a < D; ++a)
    #pragma unroll
                        for (int b = 0; b < D; ++b) mid[(ML::G + a * D + b) * cap + s] = Gb_in[a][b];
                }
                // x' = clamp(x + dt v'): no gradient through a clamped component
    #pragma unroll
                for (int a = 0; a < D; ++a) {
                    T xb = aout.x[a * cap + s];
                    T xn = xp[a] + P.dt * vn[a];
                    bool free_ = (xn >= T(0)) && (xn <= P.ext[a]);
                    xbar_c[a] = free_ ? xb : T(0);
                    const T vb_out = aout.v[a * cap + s];
                    vt_c[a] = vb_out + (free_ ? P.dt * xb : T(0));
                    if constexpr (FL) {
                        vob_c[a] = -P.flip_alpha * vb_out;
                        mid[(ML::V + a) * cap + s] = P.flip_alpha * vb_out;
                    }
    #pragma unroll
                    for (int b = 0; b < D; ++b) Lb_c[a][b] = Lb[a][b];
                }
            }
            {
                T w[D][3], dw[D][3], dd[D][3];
                int lb[3] = {0, 0, 0};
    #pragma unroll
                for (int a = 0; a < D; ++a) {
                    int b;
                    T f;
                    stencil_axis(st.x[a * cap + j], P.inv, b, f, w[a], dw[a]);
                    int l = b + g.G - tc[a] * TE;
                    lb[a] = l < 0 ? 0 : (l > TE - 1 ? TE - 1 : l);
    #pragma unroll
                    for (int q = 0; q < 3; ++q) dd[a][q] = (T(q) - f) * P.h;
                }
                T xbar[D], vt[D], Cb[D][D], Lb[D][D];
    #pragma unroll
                for (int a = 0; a < D; ++a) {
                    xbar[a] = xbar_c[a];
                    vt[a] = vt_c[a];
    #pragma unroll
                    for (int b = 0; b < D; ++b) {
                        Cb[a][b] = aout.C[(a * D + b) * cap + s];
                        Lb[a][b] = Lb_c[a][b];
                    }
                }
                // the carried matrix of the other transfers: TPIC's C' = L
                // (its adjoint joins that of L), PIC's C' = 0 (none flows back)
                if (P.xfer != XF_APIC) {
    #pragma unroll
                    for (int a = 0; a < D; ++a)
    #pragma unroll
                        for (int b = 0; b < D; ++b) {
                            if (P.xfer == XF_TPIC) Lb[a][b] += Cb[a][b];
                            Cb[a][b] = T(0);
                        }
                }
                // Line by line along x (per-axis weight factors).  Node adjoint of
                // the velocity, scattered:
                //   phi (vt + Dinv Cb dd) + Lb grad phi = w_x U + w_x dd_x V + dw_x W.
                // Position adjoint, gathered with u = Cb^T v_i, g = Lb^T v_i,
                // wbar = v_i.vt + Dinv dd.u:
                //   xbar += sum wbar grad phi + sum Hess(phi) g - Dinv Cb^T vn,
                // vn = sum phi v_i (the forward G2P velocity).
                constexpr int NL = (D == 3) ? 9 : 3;
                const T ddw[3] = {inv2, T(-2) * inv2, inv2};
                T X1[D], X2[D], vn[D];
    #pragma unroll
                for (int a = 0; a < D; ++a) { X1[a] = T(0); X2[a] = T(0); vn[a] = T(0); }
    #pragma unroll
                for (int l = 0; l < NL; ++l) {
                    const int ky = l % 3, kz = l / 3;
                    const int n0 = (D == 3) ? ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] : (lb[1] + ky) * BE + lb[0];
                    const T wy = w[1][ky], dwy = dw[1][ky];
                    const T wz = (D == 3) ? w[D - 1][kz] : T(1), dwz = (D == 3) ? dw[D - 1][kz] : T(0);
                    const T ddz = (D == 3) ? dd[D - 1][kz] : T(0);
                    const T wyz = wy * wz;
                    T U[D], V[D], Wl[D];
    #pragma unroll
                    for (int a = 0; a < D; ++a) {
                        T u = vt[a] + P.Dinv * Cb[a][1] * dd[1][ky];
                        if constexpr (D == 3) u += P.Dinv * Cb[a][D - 1] * ddz;
                        u = wyz * u + Lb[a][1] * dwy * wz;
                        if constexpr (D == 3) u += Lb[a][D - 1] * wy * dwz;
                        U[a] = u;
                        V[a] = wyz * P.Dinv * Cb[a][0];
                        Wl[a] = wyz * Lb[a][0];
                    }
                    T A = T(0), B = T(0), VN[D], Cx[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    #pragma unroll
                    for (int a = 0; a < D; ++a) VN[a] = T(0);
    #pragma unroll
                    for (int kx = 0; kx < 3; ++kx) {
                        const int n = n0 + kx;
                        const T ddn[3] = {dd[0][kx], dd[1][ky], ddz};
                        T vi[D];
    #pragma unroll
                        for (int a = 0; a < D; ++a) {
                            vi[a] = s_v[a][n];
                            T nbv = w[0][kx] * U[a] + w[0][kx] * dd[0][kx] * V[a] + dw[0][kx] * Wl[a];
                            atomicAdd(&s_b[a][n], (double)nbv);
                            if constexpr (FL) atomicAdd(&s_bo[a][n], (double)(w[0][kx] * wyz * vob_c[a]));
                        }
                        T wbar = T(0), gq[D];
    #pragma unroll
                        for (int b = 0; b < D; ++b) {
                            T ub = T(0), gb = T(0);
    #pragma unroll
                            for (int a = 0; a < D; ++a) {
                                ub += Cb[a][b] * vi[a];
                                gb += Lb[a][b] * vi[a];
                            }
                            gq[b] = gb;
                            wbar += vi[b] * vt[b] + P.Dinv * ddn[b] * ub;
                            if constexpr (FL) wbar += s_vo[b][n] * vob_c[b];
                        }
                        A += wbar * dw[0][kx];
                        B += wbar * w[0][kx];
    #pragma unroll
                        for (int a = 0; a < D; ++a) VN[a] += vi[a] * w[0][kx];
                        Cx[0] += gq[0] * ddw[kx];
                        Cx[1] += gq[1] * dw[0][kx];
                        Cx[3] += gq[0] * dw[0][kx];
                        Cx[4] += gq[1] * w[0][kx];
                        if constexpr (D == 3) {
                            Cx[2] += gq[D - 1] * dw[0][kx];
                            Cx[5] += gq[D - 1] * w[0][kx];
                        }
                    }
    #pragma unroll
                    for (int a = 0; a < D; ++a) vn[a] += wyz * VN[a];
                    if constexpr (D == 3) {
                        X1[0] += wyz * A;
                        X1[1] += dwy * wz * B;
                        X1[2] += wy * dwz * B;
                        X2[0] += wyz * Cx[0] + dwy * wz * Cx[1] + wy * dwz * Cx[2];
                        X2[1] += dwy * wz * Cx[3] + ddw[ky] * wz * Cx[4] + dwy * dwz * Cx[5];
                        X2[2] += wy * dwz * Cx[3] + dwy * dwz * Cx[4] + wy * ddw[kz] * Cx[5];
                    } else {
                        X1[0] += wy * A;
                        X1[1] += dwy * B;
                        X2[0] += wy * Cx[0] + dwy * Cx[1];
                        X2[1] += dwy * Cx[3] + ddw[ky] * Cx[4];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
    #pragma unroll
                for (int c = 0; c < D; ++c) {
                    T t = X1[c] + X2[c];
    #pragma unroll
                    for (int a = 0; a < D; ++a) t -= P.Dinv * Cb[a][c] * vn[a];
                    xbar[c] += t;
                }
    #pragma unroll
                for (int a = 0; a < D; ++a) mid[(ML::X + a) * cap + s] = xbar[a];
            }
        }
        __syncthreads();
        T* dst = part + (long long)e * NVA * NB;
        for (int i = tid; i < D * NB; i += kAdjBlock) dst[i] = (T)(&s_b[0][0])[i];
        if constexpr (FL)
            for (int i = tid; i < D * NB; i += kAdjBlock) dst[D * NB + i] = (T)(&s_bo[0][0])[i];
        __syncthreads();
    }
}

template <class T, int D>
__global__ __launch_bounds__(kAdjBlock) void k_grid_adj(Geo g, Phys<T> P, const int* __restrict__ meta,
                                                     const ActiveTile* __restrict__ active,
                                                     const int* __restrict__ tile_slot, const T* __restrict__ part,
                                                     T* __restrict__ gmass, const T* __restrict__ gvt,
                                                     T* __restrict__ gv, T* __restrict__ gvo,
                                                     double* __restrict__ amu)
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NB = TileShape<D>::NB;
    const int n_active = meta[0];
    for (int it = 0;; ++it) {
        int e = tile_entry(it, n_active);
        if (e < 0) break;
        int tile = active[e].tile;
        int tc[3];
        tile_coords(g, tile, tc);
        for (int i = threadIdx.x; i < NB; i += kAdjBlock) {
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
            // FLIP (gvo given): the partial blocks also carry the adjoint of
            // the velocity before the update, v^n = Q / m, after the first D
            const int nva = gvo ? 2 * D + 1 : D + 1;
            T vb[D], vob[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                vb[a] = T(0);
                vob[a] = T(0);
            }
            if (des == tile) {
#pragma unroll
                for (int msk = 0; msk < NC; ++msk) {
                    if (slot[msk] < 0) continue;
                    const T* src = part + (long long)slot[msk] * nva * NB;
#pragma unroll
                    for (int a = 0; a < D; ++a) vb[a] += src[a * NB + li[msk]];
                    if (gvo)
#pragma unroll
                        for (int a = 0; a < D; ++a) vob[a] += src[(D + a) * NB + li[msk]];
                }
            }
            if (des != tile) continue;
            long long node = node_index(g, I[0], I[1], I[2]);
            T m = gmass[node];
            T pb[D], mb = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) pb[a] = T(0);
            if (m > T(0)) {
                T vin[2 * D][D], vel[D];
                int nf = 0, fc[2 * D];
                T fmu[2 * D];
#pragma unroll
                for (int a = 0; a < D; ++a) vel[a] = gvt[a * g.NN + node];
                for (int a = 0; a < D; ++a) {
                    int ip = I[a] - g.G;
                    for (int side = 0; side < 2; ++side) {
                        bool beyond = side == 0 ? (ip <= 0) : (ip >= g.n[a]);
                        if (!beyond) continue;
                        int face = 2 * a + side;
                        T mu = P.wall_mu[face];
                        if (face == 2 * (D - 1) && P.floor_mu) {
                            int fx = min(I[0], g.box[0] - 1);
                            int fi = (D == 3) ? min(I[1], g.box[1] - 1) * P.floor_stride + fx : fx;
                            mu = P.floor_mu[fi];
                        }
#pragma unroll
                        for (int q = 0; q < D; ++q) vin[nf][q] = vel[q];
                        fc[nf] = face;
                        fmu[nf] = mu;
                        ++nf;
                        wall_node<T, D>(P.wall_mode[face], mu, a, side == 0 ? T(-1) : T(1), vel);
                    }
                }
                // resting obstacles after the walls (Sec. 4.2.1): a component
                // that one of them removed passes no adjoint back
                if (P.n_obst > 0) {
                    double xi[D];
#pragma unroll
                    for (int a = 0; a < D; ++a) xi[a] = double(I[a] - g.G) * P.obst_h;
                    int cut[kMaxObstacles];
                    for (int o = 0; o < P.n_obst; ++o) {
                        cut[o] = obstacle_component<T, D>(P, o, xi, vel);
                        if (cut[o] >= 0) vel[cut[o]] = T(0);
                    }
                    for (int o = P.n_obst - 1; o >= 0; --o)
                        for (int a = 0; a < D; ++a)
                            if (cut[o] == a) vb[a] = T(0);
                }
                for (int f = nf - 1; f >= 0; --f) {
                    int face = fc[f], a = face / 2;
                    T sign = (face % 2 == 0) ? T(-1) : T(1);
                    T mub = wall_node_vjp<T, D>(P.wall_mode[face], fmu[f], a, sign, vin[f], vb);
                    if (amu && face == 2 * (D - 1) && P.floor_mu && mub != T(0)) {
                        int fx = min(I[0], g.box[0] - 1);
                        int fi = (D == 3) ? min(I[1], g.box[1] - 1) * P.floor_stride + fx : fx;
                        atomicAdd(&amu[fi], (double)mub);
                    }
                }
                T dot = T(0);
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    pb[a] = vb[a] / m;
                    dot += vb[a] * (gvt[a * g.NN + node] - P.dt * P.g[a]);
                    if (gvo) dot += vob[a] * gvo[a * g.NN + node];
                }
                mb = -dot / m;
            }
#pragma unroll
            for (int a = 0; a < D; ++a) gv[a * g.NN + node] = pb[a];
            gmass[node] = mb;
            // FLIP: the adjoint of Q replaces v^n in the record
            if (gvo)
#pragma unroll
                for (int a = 0; a < D; ++a) gvo[a * g.NN + node] = m > T(0) ? vob[a] / m : T(0);
        }
    }
}

// At least two waves per SIMD: binary64 needs a few more than 256 registers
// per lane and would otherwise run one wave (measured faster with the spills).
// FLIP (FL): the force-free momentum Q (for v^n = Q / m) shares P's affine
// part, so the affine gathers take p + q (q the adjoint of Q, gqb) and the
// force's gathers p alone; the direct adjoint of v_p comes from mid.
template <class T, int D, int MAT, bool FL>
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_p2g_adj(Geo g, Phys<T> P, const int* __restrict__ meta,
                                                    const ActiveTile* __restrict__ active,
                                                    const int* __restrict__ perm, PView<T> st,
                                                    const T* __restrict__ gpb, const T* __restrict__ gmb,
                                                    const T* __restrict__ gqb,
                                                    const T* __restrict__ mid, PView<T> ain)
{
    constexpr int TE = TileShape<D>::TE, BE = TileShape<D>::BE, NB = TileShape<D>::NB;
    using ML = MidLayout<D>;
    __shared__ T s_p[D][NB];     // p (FL: p + q)
    __shared__ T s_f[FL ? D : 1][FL ? NB : 1];   // FL: p
    __shared__ T s_m[NB];
    const int n_active = meta[0];
    const int tid = threadIdx.x;
    const long long cap = st.cap;
    const T inv2 = P.inv * P.inv;
    for (int it = 0;; ++it) {
        int e = tile_entry(it, n_active);
        if (e < 0) break;
        ActiveTile at = active[e];
        int tc[3];
        tile_coords(g, at.tile, tc);
        for (int i = tid; i < NB; i += kAdjBlock) {
            int l0 = i % BE, l1 = (i / BE) % BE, l2 = (D == 3) ? i / (BE * BE) : 0;
            long long node = node_index(g, tc[0] * TE + l0, tc[1] * TE + l1, (D == 3) ? tc[2] * TE + l2 : 0);
            s_m[i] = gmb[node];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const T pv = gpb[a * g.NN + node];
                if constexpr (FL) {
                    s_f[a][i] = pv;
                    s_p[a][i] = pv + gqb[a * g.NN + node];
                } else {
                    s_p[a][i] = pv;
                }
            }
        }
        __syncthreads();
        for (int k = tid; k < at.cnt; k += kAdjBlock) {
            long long s = at.off + k;
            int j = perm[s];
            T w[D][3], dw[D][3], dd[D][3], vp[D], Cp[D][D], Sp[D][D];
            int lb[3] = {0, 0, 0};
#pragma unroll
            for (int a = 0; a < D; ++a) {
                int b;
                T f;
                stencil_axis(st.x[a * cap + j], P.inv, b, f, w[a], dw[a]);
                int l = b + g.G - tc[a] * TE;
                lb[a] = l < 0 ? 0 : (l > TE - 1 ? TE - 1 : l);
#pragma unroll
                for (int q = 0; q < 3; ++q) dd[a][q] = (T(q) - f) * P.h;
                vp[a] = st.v[a * cap + j];
#pragma unroll
                for (int b2 = 0; b2 < D; ++b2) Cp[a][b2] = st.C[(a * D + b2) * cap + j];
            }
            if constexpr (MAT == MAT_FLUID) {
                T si = st.S[j];
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) Sp[a][b] = (a == b) ? si : T(0);
            } else if constexpr (D == 3) {
                Sp[0][0] = st.S[0 * cap + j]; Sp[1][1] = st.S[1 * cap + j]; Sp[2][2] = st.S[2 * cap + j];
                Sp[0][1] = Sp[1][0] = st.S[3 * cap + j];
                Sp[0][2] = Sp[2][0] = st.S[4 * cap + j];
                Sp[1][2] = Sp[2][1] = st.S[5 * cap + j];
            } else {
                Sp[0][0] = st.S[0 * cap + j]; Sp[1][1] = st.S[1 * cap + j];
                Sp[0][1] = Sp[1][0] = st.S[2 * cap + j];
            }
            // With p_i, m_i the node adjoints of momentum and mass, the
            // particle's adjoints are gathers over its stencil:
            //   vbar = m sum phi p,  Cbar = m sum phi p (x_i - x_p)^T,
            //   Sbar = -dt sum p (grad phi)^T =: -dt Lp,
            //   xbar += m [ sum grad phi (m_i + (x_i - x_p).(Cp^T p)) + Lp^T v_p
            //              - Cp^T (sum phi p) ] - dt sum Hess(phi) (S_p p).
            T V[D], Bp[D][D], Lp[D][D], X1[D], X2[D];
            T Lf[FL ? D : 1][FL ? D : 1];   // FL: the force's sum p (grad phi)^T
#pragma unroll
            for (int a = 0; a < D; ++a) {
                V[a] = T(0);
                X1[a] = T(0);
                X2[a] = T(0);
#pragma unroll
                for (int b = 0; b < D; ++b) { Bp[a][b] = T(0); Lp[a][b] = T(0); }
            }
            if constexpr (FL)
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) Lf[a][b] = T(0);
            // Both passes run line by line along x: every weight, gradient and
            // Hessian entry of phi is a product of per-axis factors, so each
            // line is first reduced with the x factors, then combined with
            // the line's y/z factors.  ddw, the second derivative of the
            // quadratic B-spline, is (1, -2, 1)/h^2 along each axis.
            constexpr int NL = (D == 3) ? 9 : 3;
            const T ddw[3] = {inv2, T(-2) * inv2, inv2};
            T wdx[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) wdx[q] = w[0][q] * dd[0][q];
            // pass 1: the G2P-like gathers of p
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int ky = l % 3, kz = l / 3;
                const T lw = (D == 3) ? w[1][ky] * w[2][kz] : w[1][ky];
                const T ld1 = lw * dd[1][ky];
                const T ldw1 = (D == 3) ? dw[1][ky] * w[2][kz] : dw[1][ky];
                const int n0 = (D == 3) ? ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] : (lb[1] + ky) * BE + lb[0];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    T p0 = s_p[a][n0], p1 = s_p[a][n0 + 1], p2 = s_p[a][n0 + 2];
                    T A0 = w[0][0] * p0 + w[0][1] * p1 + w[0][2] * p2;
                    T A1 = wdx[0] * p0 + wdx[1] * p1 + wdx[2] * p2;
                    T A2 = dw[0][0] * p0 + dw[0][1] * p1 + dw[0][2] * p2;
                    V[a] += lw * A0;
                    Bp[a][0] += lw * A1;
                    Bp[a][1] += ld1 * A0;
                    Lp[a][0] += lw * A2;
                    Lp[a][1] += ldw1 * A0;
                    if constexpr (D == 3) {
                        Bp[a][2] += (lw * dd[2][kz]) * A0;
                        Lp[a][2] += (w[1][ky] * dw[2][kz]) * A0;
                    }
                    if constexpr (FL) {
                        T f0 = s_f[a][n0], f1 = s_f[a][n0 + 1], f2 = s_f[a][n0 + 2];
                        T F0 = w[0][0] * f0 + w[0][1] * f1 + w[0][2] * f2;
                        T F2 = dw[0][0] * f0 + dw[0][1] * f1 + dw[0][2] * f2;
                        Lf[a][0] += lw * F2;
                        Lf[a][1] += ldw1 * F0;
                        if constexpr (D == 3) Lf[a][2] += (w[1][ky] * dw[2][kz]) * F0;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            // pass 2: X1 = sum grad phi (m_i + (x_i - x_p).(Cp^T p_i)) and
            // X2 = sum Hess(phi) (S_p p_i); per node s_i and sp_i = S_p p_i,
            // per line the x-reductions
            //   A = sum s dw_x, B = sum s w_x, C1 = sum sp_x ddw_x,
            //   C2 = sum sp_y dw_x, C3 = sum sp_z dw_x, C4 = sum sp_x dw_x,
            //   C5 = sum sp_y w_x, C6 = sum sp_z w_x
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int ky = l % 3, kz = l / 3;
                const int n0 = (D == 3) ? ((lb[2] + kz) * BE + lb[1] + ky) * BE + lb[0] : (lb[1] + ky) * BE + lb[0];
                T A = T(0), B = T(0), Cx[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int n = n0 + kx;
                    T pb[D], pf[D];
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        pb[a] = s_p[a][n];
                        if constexpr (FL) pf[a] = s_f[a][n];
                        else pf[a] = pb[a];
                    }
                    T sc = s_m[n], sp[D];
                    const T ddn[3] = {dd[0][kx], dd[1][ky], (D == 3) ? dd[D - 1][kz] : T(0)};
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        T ub = T(0), sb = T(0);
#pragma unroll
                        for (int a = 0; a < D; ++a) {
                            ub += Cp[a][b] * pb[a];
                            sb += Sp[b][a] * pf[a];
                        }
                        sp[b] = sb;
                        sc += ddn[b] * ub;
                    }
                    A += sc * dw[0][kx];
                    B += sc * w[0][kx];
                    Cx[0] += sp[0] * ddw[kx];
                    Cx[1] += sp[1] * dw[0][kx];
                    Cx[3] += sp[0] * dw[0][kx];
                    Cx[4] += sp[1] * w[0][kx];
                    if constexpr (D == 3) {
                        Cx[2] += sp[D - 1] * dw[0][kx];
                        Cx[5] += sp[D - 1] * w[0][kx];
                    }
                }
                if constexpr (D == 3) {
                    const T wy = w[1][ky], dwy = dw[1][ky], wz = w[2][kz], dwz = dw[2][kz];
                    X1[0] += wy * wz * A;
                    X1[1] += dwy * wz * B;
                    X1[2] += wy * dwz * B;
                    X2[0] += wy * wz * Cx[0] + dwy * wz * Cx[1] + wy * dwz * Cx[2];
                    X2[1] += dwy * wz * Cx[3] + ddw[ky] * wz * Cx[4] + dwy * dwz * Cx[5];
                    X2[2] += wy * dwz * Cx[3] + dwy * dwz * Cx[4] + wy * ddw[kz] * Cx[5];
                } else {
                    const T wy = w[1][ky], dwy = dw[1][ky];
                    X1[0] += wy * A;
                    X1[1] += dwy * B;
                    X2[0] += wy * Cx[0] + dwy * Cx[1];
                    X2[1] += dwy * Cx[3] + ddw[ky] * Cx[4];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            T xbar[D], vbar[D], Cbar[D][D], Sbar[D][D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T t = X1[c];
#pragma unroll
                for (int a = 0; a < D; ++a) t += Lp[a][c] * vp[a] - Cp[a][c] * V[a];
                xbar[c] = mid[c * cap + s] + P.mass * t - P.dt * X2[c];
                vbar[c] = P.mass * V[c];
                if constexpr (FL) vbar[c] += mid[(ML::V + c) * cap + s];
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    Cbar[c][b] = P.mass * Bp[c][b];
                    if constexpr (FL) Sbar[c][b] = -P.dt * Lf[c][b];
                    else Sbar[c][b] = -P.dt * Lp[c][b];
                }
            }
            // the particle's adjoint goes to its slot before the step's sort
#pragma unroll
            for (int a = 0; a < D; ++a) {
                ain.x[a * cap + j] = xbar[a];
                ain.v[a * cap + j] = vbar[a];
#pragma unroll
                for (int b = 0; b < D; ++b) ain.C[(a * D + b) * cap + j] = Cbar[a][b];
            }
            if constexpr (MAT == MAT_FLUID) {
                ain.G[j] = mid[D * cap + s];
                T tr = T(0);
#pragma unroll
                for (int a = 0; a < D; ++a) tr += Sbar[a][a];
                ain.S[j] = tr;
            } else if constexpr (MAT == MAT_VFLUID) {
                // J carried; the stress is recomputed from J and L each step,
                // so its input adjoint is the force's part only
                ain.G[j] = mid[D * cap + s];
                if constexpr (D == 3) {
                    ain.S[0 * cap + j] = Sbar[0][0];
                    ain.S[1 * cap + j] = Sbar[1][1];
                    ain.S[2 * cap + j] = Sbar[2][2];
                    ain.S[3 * cap + j] = Sbar[0][1] + Sbar[1][0];
                    ain.S[4 * cap + j] = Sbar[0][2] + Sbar[2][0];
                    ain.S[5 * cap + j] = Sbar[1][2] + Sbar[2][1];
                } else {
                    ain.S[0 * cap + j] = Sbar[0][0];
                    ain.S[1 * cap + j] = Sbar[1][1];
                    ain.S[2 * cap + j] = Sbar[0][1] + Sbar[1][0];
                }
            } else if constexpr (MAT == MAT_JAUMANN) {
                // the force's part of the stress adjoint plus the constitutive part
                constexpr int S0 = MidLayout<D>::S;
                ain.G[j] = mid[D * cap + s];
                if constexpr (D == 3) {
                    ain.S[0 * cap + j] = Sbar[0][0] + mid[(S0 + 0) * cap + s];
                    ain.S[1 * cap + j] = Sbar[1][1] + mid[(S0 + 1) * cap + s];
                    ain.S[2 * cap + j] = Sbar[2][2] + mid[(S0 + 2) * cap + s];
                    ain.S[3 * cap + j] = Sbar[0][1] + Sbar[1][0] + mid[(S0 + 3) * cap + s];
                    ain.S[4 * cap + j] = Sbar[0][2] + Sbar[2][0] + mid[(S0 + 4) * cap + s];
                    ain.S[5 * cap + j] = Sbar[1][2] + Sbar[2][1] + mid[(S0 + 5) * cap + s];
                } else {
                    ain.S[0 * cap + j] = Sbar[0][0] + mid[(S0 + 0) * cap + s];
                    ain.S[1 * cap + j] = Sbar[1][1] + mid[(S0 + 1) * cap + s];
                    ain.S[2 * cap + j] = Sbar[0][1] + Sbar[1][0] + mid[(S0 + 2) * cap + s];
                }
            } else {
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) ain.G[(a * D + b) * cap + j] = mid[(D + a * D + b) * cap + s];
                if constexpr (D == 3) {
                    ain.S[0 * cap + j] = Sbar[0][0];
                    ain.S[1 * cap + j] = Sbar[1][1];
                    ain.S[2 * cap + j] = Sbar[2][2];
                    ain.S[3 * cap + j] = Sbar[0][1] + Sbar[1][0];
                    ain.S[4 * cap + j] = Sbar[0][2] + Sbar[2][0];
                    ain.S[5 * cap + j] = Sbar[1][2] + Sbar[2][1];
                } else {
                    ain.S[0 * cap + j] = Sbar[0][0];
                    ain.S[1 * cap + j] = Sbar[1][1];
                    ain.S[2 * cap + j] = Sbar[0][1] + Sbar[1][0];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Observation operators and loss (Sec. 3.2, eq:inverse_loss)
// ---------------------------------------------------------------------------

template <int Unused = 0>
__global__ void k_inverse_pid(const int32_t* __restrict__ pid, long long N, int32_t* __restrict__ inv)
{
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s < N) inv[pid[s]] = (int32_t)s;
}

// Lagrangian tracers: Q_l = z of particle l.  Adds m |Q - z_obs|^2 to the
// loss and, when seed != 0, 2 m (Q - z_obs) to the adjoint of z.
template <class T, int D>
__global__ void k_lag_obs(const T* __restrict__ z, T* __restrict__ zb, long long cap, long long N,
                          const int32_t* __restrict__ inv, const int32_t* __restrict__ tracer, int ntr,
                          const T* __restrict__ target, const T* __restrict__ mask, int seed,
                          double* __restrict__ loss)
{
    int l = blockIdx.x * kBlock + threadIdx.x;
    double part = 0.0;
    // an id outside [0, N) is skipped (it names no particle)
    if (l < ntr && tracer[l] >= 0 && tracer[l] < N) {
        int s = inv[tracer[l]];
        T m = mask ? mask[l] : T(1);
        if (m != T(0)) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                T r = z[a * cap + s] - target[a * ntr + l];
                part += (double)m * (double)r * (double)r;
                if (seed) zb[a * cap + s] += T(2) * m * r;
            }
        }
    }
    // wave reduction, one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((threadIdx.x & 63) == 0 && part != 0.0) atomicAdd(loss, part);
}

struct Boxes {
    double lo[kMaxBoxes][3], hi[kMaxBoxes][3];
    int n;
};

template <class T, int D>
__device__ __forceinline__ bool in_box(const Boxes& bx, int b, const T* x, long long cap, long long s)
{
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T xv = x[a * cap + s];
        in = in && (xv >= (T)bx.lo[b][a]) && (xv < (T)bx.hi[b][a]);
    }
    return in;
}

// Eulerian boxes, pass 1: per-box sums of z and particle counts (binary64).
template <class T, int D>
__global__ void k_box_sum(Boxes bx, const T* __restrict__ x, const T* __restrict__ z, long long cap, long long N,
                          double* __restrict__ sum, int* __restrict__ cnt)
{
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    for (int b = 0; b < bx.n; ++b) {
        bool in = s < N && in_box<T, D>(bx, b, x, cap, s);
        unsigned long long msk = __ballot(in);
        double acc[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double v = in ? (double)z[a * cap + s] : 0.0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            acc[a] = v;
        }
        if ((threadIdx.x & 63) == 0 && msk) {
            atomicAdd(&cnt[b], __popcll(msk));
#pragma unroll
            for (int a = 0; a < D; ++a) atomicAdd(&sum[b * 3 + a], acc[a]);
        }
    }
}

// Eulerian boxes, pass 2 (one thread per box): Q, the loss and the seed
// coefficient 2 m (Q - z_obs) / |P_l| per box; empty boxes contribute nothing.
template <class T, int D>
__global__ void k_box_loss(int nbox, const double* __restrict__ sum, const int* __restrict__ cnt,
                           const T* __restrict__ target, const T* __restrict__ mask, double* __restrict__ coef,
                           double* __restrict__ loss)
{
    int b = threadIdx.x;
    if (b >= nbox) return;
    double m = mask ? (double)mask[b] : 1.0;
    int c = cnt[b];
    double part = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double cf = 0.0;
        if (c > 0 && m != 0.0) {
            double r = sum[b * 3 + a] / c - (double)target[a * nbox + b];
            part += m * r * r;
            cf = 2.0 * m * r / c;
        }
        coef[b * 3 + a] = cf;
    }
    if (part != 0.0) atomicAdd(loss, part);
}

template <class T, int D>
__global__ void k_box_seed(Boxes bx, const T* __restrict__ x, T* __restrict__ zb, long long cap, long long N,
                           const double* __restrict__ coef)
{
    long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    for (int b = 0; b < bx.n; ++b) {
        if (!in_box<T, D>(bx, b, x, cap, s)) continue;
#pragma unroll
        for (int a = 0; a < D; ++a) zb[a * cap + s] += (T)coef[b * 3 + a];
    }
}

template <class T, int D>
__global__ void k_lag_extract(const T* __restrict__ z, long long cap, long long N, const int32_t* __restrict__ inv,
                              const int32_t* __restrict__ tracer, int ntr, T* __restrict__ q)
{
    int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= ntr) return;
    int id = tracer[l];
    bool ok = id >= 0 && id < N;
    int s = ok ? inv[id] : 0;
#pragma unroll
    for (int a = 0; a < D; ++a) q[a * ntr + l] = ok ? z[a * cap + s] : T(0);
}

template <class T, int D>
__global__ void k_box_mean(int nbox, const double* __restrict__ sum, const int* __restrict__ cnt, T* __restrict__ q)
{
    int b = threadIdx.x;
    if (b >= nbox) return;
#pragma unroll
    for (int a = 0; a < D; ++a) q[a * nbox + b] = cnt[b] > 0 ? (T)(sum[b * 3 + a] / cnt[b]) : T(0);
}

template <class T>
__global__ void k_mu_out(const double* __restrict__ amu, long long n, T* __restrict__ out)
{
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = (T)amu[i];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

template <class T, int D>
struct Adjoint {
    using S = Solver<T, D>;

    static PView<T> slot_view(const mpm_ctx* c, char* base, int32_t* pid)
    {
        PView<T> v{};
        T* b = (T*)base;
        long long cap = c->cap;
        v.cap = cap;
        v.x = b;
        v.v = b + D * cap;
        v.C = b + 2 * D * cap;
        v.G = b + (2 * D + D * D) * cap;
        v.S = v.G + (mat_has_F(c->mat) ? D * D : 1) * cap;
        v.pid = pid;
        return v;
    }
    static size_t state_bytes(const mpm_ctx* c) { return (size_t)c->nsc * (size_t)c->cap * sizeof(T); }
    static PView<T> ckpt(const mpm_ctx* c, int i)
    {
        return slot_view(c, c->ckpt + (size_t)i * state_bytes(c), c->ckpt_pid + (size_t)i * c->cap);
    }
    // State i (0..ckpt_every) of tape slot q (one slot per taped segment).
    static PView<T> tape(const mpm_ctx* c, int q, int i)
    {
        const size_t at = (size_t)q * (size_t)(c->ckpt_every + 1) + (size_t)i;
        return slot_view(c, c->tape + at * state_bytes(c), c->tape_pid + at * c->cap);
    }
    static PView<T> adj(const mpm_ctx* c, int i) { return slot_view(c, c->adj[i], nullptr); }

    static int copy_state(mpm_ctx* c, const PView<T>& dst, const PView<T>& src)
    {
        hipStream_t st = c->stream;
        if (hipMemcpyAsync(dst.x, src.x, state_bytes(c), hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(dst.pid, src.pid, sizeof(int32_t) * c->cap, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return S::launch_err(c, "state copy");
        return MPM_OK;
    }

    static void keys_of(mpm_ctx* c, const PView<T>& v)
    {
        hipStream_t st = c->stream;
        k_fill<int><<<std::min<long long>(nblocks(c->geo.ntiles), 4096), kBlock, 0, st>>>(c->count, c->geo.ntiles, 0);
        Phys<T> P = make_phys<T>(c, 0.0);
        k_keys<T, D><<<nblocks(c->N), kBlock, 0, st>>>(c->geo, P, v, c->N, c->key, c->count);
    }

    // The grid-tape record of step i of the segment in tape slot q.
    static typename S::StepBufs rec_bufs(const mpm_ctx* c, int q, int i)
    {
        char* r = c->gtape + ((size_t)q * (size_t)c->ckpt_every + (size_t)i) * c->grec.bytes;
        return {(int32_t*)(r + c->grec.perm), (int32_t*)(r + c->grec.tile_slot), (ActiveTile*)(r + c->grec.active),
                (int32_t*)(r + c->grec.meta), (T*)(r + c->grec.gv), (T*)(r + c->grec.gmass),
                (T*)(r + c->grec.gvt), c->xfer == XF_FLIP ? (T*)(r + c->grec.gvo) : nullptr};
    }

    // Reverse of one step whose sort and grid are in record rb (written by
    // the segment's forward recomputation): aout holds the adjoint of the
    // step's output state, ain receives that of its input state st_in.  The
    // record's nodal velocity and mass are overwritten by their adjoints.
    template <int MAT>
    static void adjoint_step(mpm_ctx* c, const Phys<T>& P, const PView<T>& st_in, const PView<T>& aout,
                             const PView<T>& ain, const typename S::StepBufs& rb)
    {
        hipStream_t st = c->stream;
        const Geo& g = c->geo;
        prof_mark(c, -1);
        const bool flip = c->xfer == XF_FLIP;
        if (flip)
            k_g2p_adj<T, D, MAT, true><<<kTileWGs * kBlock / kAdjBlock, kAdjBlock, 0, st>>>(
                g, P, rb.meta, rb.active, rb.perm, st_in, aout, (const T*)rb.gv, (const T*)rb.gvo, (T*)c->part_grid,
                (T*)c->mid);
        else
            k_g2p_adj<T, D, MAT, false><<<kTileWGs * kBlock / kAdjBlock, kAdjBlock, 0, st>>>(
                g, P, rb.meta, rb.active, rb.perm, st_in, aout, (const T*)rb.gv, nullptr, (T*)c->part_grid,
                (T*)c->mid);
        prof_mark(c, MPM_PROF_G2P_ADJ);
        k_grid_adj<T, D><<<kTileWGs * kBlock / kAdjBlock, kAdjBlock, 0, st>>>(g, P, rb.meta, rb.active, rb.tile_slot,
                                                      (const T*)c->part_grid, rb.gmass, (const T*)rb.gvt, rb.gv,
                                                      flip ? rb.gvo : nullptr, c->floor_mu ? c->amu : nullptr);
        prof_mark(c, MPM_PROF_GRID_ADJ);
        if (flip)
            k_p2g_adj<T, D, MAT, true><<<kTileWGs * kBlock / kAdjBlock, kAdjBlock, 0, st>>>(
                g, P, rb.meta, rb.active, rb.perm, st_in, (const T*)rb.gv, (const T*)rb.gmass, (const T*)rb.gvo,
                (const T*)c->mid, ain);
        else
            k_p2g_adj<T, D, MAT, false><<<kTileWGs * kBlock / kAdjBlock, kAdjBlock, 0, st>>>(
                g, P, rb.meta, rb.active, rb.perm, st_in, (const T*)rb.gv, (const T*)rb.gmass, nullptr,
                (const T*)c->mid, ain);
        prof_mark(c, MPM_PROF_P2G_ADJ);
    }

    static Boxes boxes(const mpm_ctx* c)
    {
        Boxes b{};
        b.n = c->obs_nbox;
        for (int i = 0; i < b.n; ++i)
            for (int a = 0; a < 3; ++a) {
                b.lo[i][a] = c->box_lo[i][a];
                b.hi[i][a] = c->box_hi[i][a];
            }
        return b;
    }

    // Loss of frame fi on state v; with zb_* non-null also the seeds.
    static void observe(mpm_ctx* c, const PView<T>& v, int fi, const PView<T>* ab)
    {
        hipStream_t st = c->stream;
        long long N = c->N;
        if (c->obs_ntr > 0) {
            k_inverse_pid<0><<<nblocks(N), kBlock, 0, st>>>(v.pid, N, c->inv);
            const T* z = c->obs_lag_field == MPM_FIELD_X ? v.x : v.v;
            T* zb = ab ? (c->obs_lag_field == MPM_FIELD_X ? ab->x : ab->v) : nullptr;
            const T* tgt = (const T*)c->obs_lag_target + (size_t)fi * D * c->obs_ntr;
            const T* msk = c->obs_lag_mask ? (const T*)c->obs_lag_mask + (size_t)fi * c->obs_ntr : nullptr;
            k_lag_obs<T, D><<<nblocks(c->obs_ntr), kBlock, 0, st>>>(z, zb, v.cap, N, c->inv, c->obs_tracer,
                                                                    c->obs_ntr, tgt, msk, ab ? 1 : 0, c->loss);
        }
        if (c->obs_nbox > 0) {
            Boxes bx = boxes(c);
            k_fill<double><<<1, kBlock, 0, st>>>(c->box_sum, kMaxBoxes * 3, 0.0);
            k_fill<int><<<1, kBlock, 0, st>>>(c->box_cnt, kMaxBoxes, 0);
            const T* z = c->obs_eul_field == MPM_FIELD_X ? v.x : v.v;
            k_box_sum<T, D><<<nblocks(N), kBlock, 0, st>>>(bx, v.x, z, v.cap, N, c->box_sum, c->box_cnt);
            const T* tgt = (const T*)c->obs_eul_target + (size_t)fi * D * c->obs_nbox;
            const T* msk = c->obs_eul_mask ? (const T*)c->obs_eul_mask + (size_t)fi * c->obs_nbox : nullptr;
            // the seed pass must not add this frame's loss twice
            double* loss_dst = ab ? c->loss_scratch : c->loss;
            k_box_loss<T, D><<<1, kMaxBoxes, 0, st>>>(c->obs_nbox, c->box_sum, c->box_cnt, tgt, msk, c->box_coef,
                                                      loss_dst);
            if (ab) {
                T* zb = c->obs_eul_field == MPM_FIELD_X ? ab->x : ab->v;
                k_box_seed<T, D><<<nblocks(N), kBlock, 0, st>>>(bx, v.x, zb, v.cap, N, c->box_coef);
            }
        }
    }

    static int frame_index(const mpm_ctx* c, int t)
    {
        for (size_t i = 0; i < c->obs_frames.size(); ++i)
            if (c->obs_frames[i] == t) return (int)i;
        return -1;
    }

    template <int MAT, int XF>
    static int forward_loss_mat(mpm_ctx* c, int n, double dt, double* loss)
    {
        hipStream_t st = c->stream;
        Phys<T> P = make_phys<T>(c, dt);
        Phys<T> Pk = P;
        Pk.keep_grid = 1;
        const int k = c->ckpt_every;
        // the trailing tape_segs segments run directly on the tape (states
        // and grid records), so the backward sweep reverses them without
        // recomputing them
        const int nseg = (n + k - 1) / k;
        const int nt = std::max(1, std::min(c->tape_segs, nseg));
        const int first = nseg - nt, tl = first * k;
        c->taped = 0;
        k_fill<double><<<1, kBlock, 0, st>>>(c->loss, 2, 0.0);
        for (int t = 0; t < n; ++t) {
            if (t % k == 0) {
                // the state at t: in the context up to the first taped
                // segment, then at the end of the previous taped segment
                const PView<T> now = t <= tl ? view<T>(c, c->cur) : tape(c, t / k - first - 1, k);
                int rc = copy_state(c, ckpt(c, t / k), now);
                if (rc) return rc;
            }
            PView<T> obs_state;
            if (t < tl) {
                PView<T> cur = view<T>(c, c->cur), nxt = view<T>(c, 1 - c->cur);
                S::template step_views<MAT, XF>(c, P, cur, nxt);
                c->cur = 1 - c->cur;
                obs_state = view<T>(c, c->cur);
            } else {
                const int q = t / k - first, i = t - (t / k) * k;
                if (i == 0) {
                    int rc = copy_state(c, tape(c, q, 0), q == 0 ? view<T>(c, c->cur) : tape(c, q - 1, k));
                    if (rc) return rc;
                }
                S::template step_views<MAT, XF>(c, Pk, tape(c, q, i), tape(c, q, i + 1), rec_bufs(c, q, i));
                obs_state = tape(c, q, i + 1);
            }
            int fi = frame_index(c, t + 1);
            if (fi >= 0) observe(c, obs_state, fi, nullptr);
        }
        // the context's state, sort and grid again describe the last step
        {
            const int ql = nt - 1, il = n - (nseg - 1) * k;
            int rc = copy_state(c, view<T>(c, c->cur), tape(c, ql, il));
            if (rc) return rc;
            typename S::StepBufs last = rec_bufs(c, ql, il - 1);
            const size_t nn = (size_t)c->geo.NN * sizeof(T);
            rc = hip_check(c, hipMemcpyAsync(c->perm, last.perm, (size_t)c->cap * 4, hipMemcpyDeviceToDevice, st),
                           "sort copy");
            if (!rc) rc = hip_check(c, hipMemcpyAsync(c->gv, last.gv, D * nn, hipMemcpyDeviceToDevice, st), "grid copy");
            if (!rc)
                rc = hip_check(c, hipMemcpyAsync(c->tile_slot, last.tile_slot, (size_t)c->geo.ntiles * 4,
                                                 hipMemcpyDeviceToDevice, st), "grid copy");
            if (!rc && c->cfg.keep_grid)
                rc = hip_check(c, hipMemcpyAsync(c->gmass, last.gmass, nn, hipMemcpyDeviceToDevice, st), "grid copy");
            if (rc) return rc;
        }
        c->taped = nt;
        int rc = S::launch_err(c, "forward loss");
        if (rc) return rc;
        double h[2];
        rc = hip_check(c, hipMemcpyAsync(h, c->loss, sizeof(h), hipMemcpyDeviceToHost, st), "loss read");
        if (rc) return rc;
        rc = hip_check(c, hipStreamSynchronize(st), "stream synchronize");
        if (rc) return rc;
        *loss = h[0];
        return MPM_OK;
    }

    template <int MAT, int XF>
    static int backward_mat(mpm_ctx* c, void* grad_v0, void* grad_mu)
    {
        hipStream_t st = c->stream;
        const int n = c->fwd_steps, k = c->ckpt_every;
        Phys<T> P = make_phys<T>(c, c->fwd_dt);
        Phys<T> Pk = P;   // the recomputed steps keep their nodal mass
        Pk.keep_grid = 1;
        int a = 0;   // adjoint buffer holding the adjoint of the later state
        k_fill<T><<<4096, kBlock, 0, st>>>((T*)c->adj[0], (long long)c->nsc * c->cap, T(0));
        long long nfl = c->geo.dim == 3 ? (long long)c->geo.box[0] * c->geo.box[1] : c->geo.box[0];
        k_fill<double><<<std::min<long long>(nblocks(nfl), 4096), kBlock, 0, st>>>(c->amu, nfl, 0.0);
        const int nseg = (n + k - 1) / k;
        // the forward pass left its trailing segments on the tape (once: the
        // reverse steps overwrite the grid records with adjoints); earlier
        // segments are recomputed from their checkpoint into slot 0, which the
        // taped segments have released by then
        const int first = nseg - c->taped;
        c->taped = 0;
        for (int seg = nseg - 1; seg >= 0; --seg) {
            int t0 = seg * k, t1 = std::min(t0 + k, n);
            const bool on_tape = seg >= first;
            const int q = on_tape ? seg - first : 0;
            if (!on_tape) {
                int rc = copy_state(c, tape(c, 0, 0), ckpt(c, seg));
                if (rc) return rc;
                keys_of(c, tape(c, 0, 0));
                for (int t = t0; t < t1; ++t)
                    S::template step_views<MAT, XF>(c, Pk, tape(c, 0, t - t0), tape(c, 0, t - t0 + 1),
                                                    rec_bufs(c, 0, t - t0));
            }
            for (int t = t1 - 1; t >= t0; --t) {
                int fi = frame_index(c, t + 1);
                PView<T> aout = adj(c, a), ain = adj(c, 1 - a);
                if (fi >= 0) observe(c, tape(c, q, t + 1 - t0), fi, &aout);
                adjoint_step<MAT>(c, P, tape(c, q, t - t0), aout, ain, rec_bufs(c, q, t - t0));
                a = 1 - a;
            }
        }
        // dL/dv0 in pid order (S^0 is checkpoint 0)
        if (grad_v0 && c->N > 0)
            k_read_field<T, D><<<nblocks(c->N), kBlock, 0, st>>>(adj(c, a).v, c->cap, ckpt(c, 0).pid, c->N, D,
                                                                CONV_COPY, 1, (T*)grad_v0);
        if (grad_mu) k_mu_out<T><<<nblocks(nfl), kBlock, 0, st>>>(c->amu, nfl, (T*)grad_mu);
        // the step's key and count arrays again describe the current state
        int rc = S::recompute_keys(c);
        if (rc) return rc;
        rc = S::launch_err(c, "backward");
        if (rc) return rc;
        return hip_check(c, hipStreamSynchronize(st), "stream synchronize");
    }

    static int extract(mpm_ctx* c, void* lag_q, void* eul_q)
    {
        hipStream_t st = c->stream;
        PView<T> v = view<T>(c, c->cur);
        long long N = c->N;
        if (lag_q && c->obs_ntr > 0) {
            k_inverse_pid<0><<<nblocks(N), kBlock, 0, st>>>(v.pid, N, c->inv);
            const T* z = c->obs_lag_field == MPM_FIELD_X ? v.x : v.v;
            k_lag_extract<T, D><<<nblocks(c->obs_ntr), kBlock, 0, st>>>(z, v.cap, N, c->inv, c->obs_tracer,
                                                                        c->obs_ntr, (T*)lag_q);
        }
        if (eul_q && c->obs_nbox > 0) {
            Boxes bx = boxes(c);
            k_fill<double><<<1, kBlock, 0, st>>>(c->box_sum, kMaxBoxes * 3, 0.0);
            k_fill<int><<<1, kBlock, 0, st>>>(c->box_cnt, kMaxBoxes, 0);
            const T* z = c->obs_eul_field == MPM_FIELD_X ? v.x : v.v;
            k_box_sum<T, D><<<nblocks(N), kBlock, 0, st>>>(bx, v.x, z, v.cap, N, c->box_sum, c->box_cnt);
            k_box_mean<T, D><<<1, kMaxBoxes, 0, st>>>(c->obs_nbox, c->box_sum, c->box_cnt, (T*)eul_q);
        }
        return S::launch_err(c, "extract");
    }

    // the reverse sweep of each transfer
    template <int MAT>
    static int forward_loss_x(mpm_ctx* c, int n, double dt, double* loss)
    {
        switch (c->xfer) {
        case XF_PIC: return forward_loss_mat<MAT, XF_PIC>(c, n, dt, loss);
        case XF_TPIC: return forward_loss_mat<MAT, XF_TPIC>(c, n, dt, loss);
        case XF_FLIP: return forward_loss_mat<MAT, XF_FLIP>(c, n, dt, loss);
        default: return forward_loss_mat<MAT, XF_APIC>(c, n, dt, loss);
        }
    }
    template <int MAT>
    static int backward_x(mpm_ctx* c, void* gv0, void* gmu)
    {
        switch (c->xfer) {
        case XF_PIC: return backward_mat<MAT, XF_PIC>(c, gv0, gmu);
        case XF_TPIC: return backward_mat<MAT, XF_TPIC>(c, gv0, gmu);
        case XF_FLIP: return backward_mat<MAT, XF_FLIP>(c, gv0, gmu);
        default: return backward_mat<MAT, XF_APIC>(c, gv0, gmu);
        }
    }
    static int forward_loss(mpm_ctx* c, int n, double dt, double* loss)
    {
        switch (c->mat) {
        case MAT_FLUID: return forward_loss_x<MAT_FLUID>(c, n, dt, loss);
        case MAT_VFLUID: return forward_loss_x<MAT_VFLUID>(c, n, dt, loss);
        case MAT_JAUMANN: return forward_loss_x<MAT_JAUMANN>(c, n, dt, loss);
        case MAT_SAND: return forward_loss_x<MAT_SAND>(c, n, dt, loss);
        default: return forward_loss_x<MAT_ELASTIC>(c, n, dt, loss);
        }
    }
    static int backward(mpm_ctx* c, void* gv0, void* gmu)
    {
        switch (c->mat) {
        case MAT_FLUID: return backward_x<MAT_FLUID>(c, gv0, gmu);
        case MAT_VFLUID: return backward_x<MAT_VFLUID>(c, gv0, gmu);
        case MAT_JAUMANN: return backward_x<MAT_JAUMANN>(c, gv0, gmu);
        case MAT_SAND: return backward_x<MAT_SAND>(c, gv0, gmu);
        default: return backward_x<MAT_ELASTIC>(c, gv0, gmu);
        }
    }
};

}  // namespace mpm
