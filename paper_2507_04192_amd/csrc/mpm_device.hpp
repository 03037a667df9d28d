// Device-side building blocks of the MPM step for gfx950: quadratic B-spline
// stencil, small symmetric eigen-solver, constitutive updates, wall rules and
// wave-level helpers.  Templated on the working precision T (float/double)
// and the dimension D (2/3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm_types.hpp"

namespace mpm {

// ---------------------------------------------------------------------------
// Scalar helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float mul_exact(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_exact(double a, double b) { return __dmul_rn(a, b); }

template <class T> __device__ __forceinline__ T sq(T a) { return a * a; }

template <class T> __device__ __forceinline__ bool finite(T a) { return isfinite(a); }

// ---------------------------------------------------------------------------
// Quadratic B-spline stencil (Sec. 2.1).  For t = x/h (rounded product,
// never fused) the base node is b = floor(t - 1/2) and f = t - b lies in
// [1/2, 3/2); node b+k has xi = f - k.  The three weights are the pieces of
// phi-bar evaluated there, and dw is d phi / dx.
// ---------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ void stencil_axis(T x, T inv, int& b, T& f, T w[3], T dw[3])
{
    T t = mul_exact(x, inv);
    T fb = floor(t - T(0.5));
    b = (int)fb;
    f = t - fb;
    T a0 = T(1.5) - f, a1 = f - T(1), a2 = f - T(0.5);
    w[0] = T(0.5) * a0 * a0;
    w[1] = T(0.75) - a1 * a1;
    w[2] = T(0.5) * a2 * a2;
    dw[0] = -a0 * inv;
    dw[1] = T(-2) * a1 * inv;
    dw[2] = a2 * inv;
}

template <class T>
__device__ __forceinline__ int base_of(T x, T inv)
{
    T t = mul_exact(x, inv);
    return (int)floor(t - T(0.5));
}

// ---------------------------------------------------------------------------
// Cell key: tile-major linear index of the base node (base + ghost), tiles
// ordered x fastest, then the cells inside a tile x fastest.  Every tile has
// 64 cells (4^3 in 3D, 8^2 in 2D), so key >> 6 is the tile and key & 63 the
// cell inside it.
// ---------------------------------------------------------------------------

template <class T, int D>
__device__ __forceinline__ int cell_key(const Geo& g, const T* xp, T inv)
{
    // the tile edge is 4 cells in 3-D and 8 in 2-D (the configuration check
    // admits no other), so the tile and cell coordinates are a shift and a mask
    constexpr int TE = (D == 3) ? 4 : 8, SH = (D == 3) ? 2 : 3;
    int tl = 0, cl = 0, ts = 1, cs = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        int B = base_of(xp[a], inv) + g.G;
        B = B < 0 ? 0 : (B > g.bmax[a] ? g.bmax[a] : B);   // memory guard only
        tl += (B >> SH) * ts;
        cl += (B & (TE - 1)) * cs;
        ts *= g.ntile[a];
        cs *= TE;
    }
    return tl * 64 + cl;
}

// Tile coordinates of a tile index.
__device__ __forceinline__ void tile_coords(const Geo& g, int tile, int tc[3])
{
    tc[0] = tile % g.ntile[0];
    int r = tile / g.ntile[0];
    tc[1] = r % g.ntile[1];
    tc[2] = r / g.ntile[1];
}

__device__ __forceinline__ long long node_index(const Geo& g, int I0, int I1, int I2)
{
    return ((long long)I2 * g.nd[1] + I1) * g.nd[0] + I0;
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Groups consecutive lanes holding the same value v (valid lanes only) into
// runs.  Returns the run's first lane, its length and this lane's rank.
__device__ __forceinline__ void wave_runs(int v, bool valid, int& head_lane, int& run_len, int& rank)
{
    int lane = lane_id();
    int prev = __shfl_up(v, 1);
    int prev_valid = __shfl_up((int)valid, 1);
    bool head = valid && (lane == 0 || !prev_valid || prev != v);
    unsigned long long heads = __ballot(head);
    unsigned long long le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    unsigned long long mine = heads & le;
    head_lane = 63 - __clzll(mine ? mine : 1ull);
    unsigned long long above = heads & ~le;
    unsigned long long vmask = __ballot(valid);
    int next_head = above ? (__ffsll((long long)above) - 1) : 64;
    // a run ends at the next head or at the first invalid lane after it
    unsigned long long inval_above = ~vmask & ~le;
    int next_inval = inval_above ? (__ffsll((long long)inval_above) - 1) : 64;
    int end = next_head < next_inval ? next_head : next_inval;
    run_len = end - head_lane;
    rank = lane - head_lane;
}

// ---------------------------------------------------------------------------
// Symmetric eigen-decomposition by cyclic Jacobi rotations, in registers.
// A = V diag(ev) V^T.  Packed input: 3D (a00,a11,a22,a01,a02,a12);
// 2D (a00,a11,a01).  Float stops after a fixed sweep budget; double iterates
// until the off-diagonal part is negligible and returns false if the sweep
// budget ran out first (float always returns true).
// ---------------------------------------------------------------------------

template <class T> struct JacobiTol;
template <> struct JacobiTol<float> { static constexpr int sweeps = 6; static constexpr float rel = 1e-14f; static constexpr float big = 1e7f; };
template <> struct JacobiTol<double> { static constexpr int sweeps = 12; static constexpr double rel = 1e-32; static constexpr double big = 1e15; };

template <class T>
__device__ __forceinline__ void jacobi_rot(T& app, T& aqq, T& apq, T& c, T& s)
{
    T theta = (aqq - app) / (T(2) * apq);
    T at = fabs(theta);
    T t = (at > JacobiTol<T>::big) ? T(0.5) / theta
                                   : copysign(T(1), theta) / (at + sqrt(theta * theta + T(1)));
    c = T(1) / sqrt(t * t + T(1));
    s = t * c;
    app -= t * apq;
    aqq += t * apq;
    apq = T(0);
}

template <class T>
__device__ __forceinline__ bool sym_eig3(const T a_in[6], T ev[3], T V[3][3])
{
    T a00 = a_in[0], a11 = a_in[1], a22 = a_in[2], a01 = a_in[3], a02 = a_in[4], a12 = a_in[5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? T(1) : T(0);
    for (int sw = 0; sw < JacobiTol<T>::sweeps; ++sw) {
        T off = a01 * a01 + a02 * a02 + a12 * a12;
        T dia = a00 * a00 + a11 * a11 + a22 * a22;
        if (off <= JacobiTol<T>::rel * dia || off == T(0)) break;
        T c, s;
        // (p,q) = (0,1), r = 2
        if (a01 != T(0)) {
            jacobi_rot(a00, a11, a01, c, s);
            T r0 = a02, r1 = a12;
            a02 = c * r0 - s * r1;
            a12 = s * r0 + c * r1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T vp = V[k][0], vq = V[k][1];
                V[k][0] = c * vp - s * vq;
                V[k][1] = s * vp + c * vq;
            }
        }
        // (p,q) = (0,2), r = 1
        if (a02 != T(0)) {
            jacobi_rot(a00, a22, a02, c, s);
            T r0 = a01, r1 = a12;
            a01 = c * r0 - s * r1;
            a12 = s * r0 + c * r1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T vp = V[k][0], vq = V[k][2];
                V[k][0] = c * vp - s * vq;
                V[k][2] = s * vp + c * vq;
            }
        }
        // (p,q) = (1,2), r = 0
        if (a12 != T(0)) {
            jacobi_rot(a11, a22, a12, c, s);
            T r0 = a01, r1 = a02;
            a01 = c * r0 - s * r1;
            a02 = s * r0 + c * r1;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T vp = V[k][1], vq = V[k][2];
                V[k][1] = c * vp - s * vq;
                V[k][2] = s * vp + c * vq;
            }
        }
    }
    ev[0] = a00;
    ev[1] = a11;
    ev[2] = a22;
    if constexpr (sizeof(T) == 4) return true;
    T off = a01 * a01 + a02 * a02 + a12 * a12;
    return off <= JacobiTol<T>::rel * (a00 * a00 + a11 * a11 + a22 * a22);
}

template <class T>
__device__ __forceinline__ void sym_eig2(const T a_in[3], T ev[2], T V[2][2])
{
    T a00 = a_in[0], a11 = a_in[1], a01 = a_in[2];
    T c = T(1), s = T(0);
    if (a01 != T(0)) jacobi_rot(a00, a11, a01, c, s);
    V[0][0] = c;  V[0][1] = s;
    V[1][0] = -s; V[1][1] = c;
    ev[0] = a00;
    ev[1] = a11;
}

// Hencky strain magnitude |eps|_F at or below which the Drucker-Prager
// return takes the elastic case whatever the sign of tr(eps).  The return is
// not differentiable at zero strain; this fixes the case there (a body at
// rest, whose strain is rounding noise) instead of leaving it to rounding.
// The resulting stress is at most E times this strain.
template <class T> __device__ __forceinline__ constexpr T eps_elastic2() { return T(1e-12); }

// ---------------------------------------------------------------------------
// Constitutive updates.  S is V0 * Kirchhoff stress (= V_p sigma_p), stored
// symmetric: 3D (xx,yy,zz,xy,xz,yz), 2D (xx,yy,xy); a fluid stores the single
// isotropic value s with S = s I.
// ---------------------------------------------------------------------------

// Fluid: J' = J det(I + dt L), p = (K/gamma)((1/J')^gamma - 1), S = -V0 J' p I.
// Uses dJ = J - 1 and det(I + A) - 1 expanded in the invariants of A so that
// small volume changes keep their relative accuracy.
template <class T, int D>
__device__ __forceinline__ void fluid_update(const Phys<T>& P, const T L[D][D], T& dJ, T& s_iso)
{
    T dt = P.dt;
    T dD;
    if constexpr (D == 3) {
        T A[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[i][j] = dt * L[i][j];
        T tr = A[0][0] + A[1][1] + A[2][2];
        T m2 = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) + (A[0][0] * A[2][2] - A[0][2] * A[2][0]) +
               (A[1][1] * A[2][2] - A[1][2] * A[2][1]);
        T det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        dD = tr + m2 + det;
    } else {
        T a00 = dt * L[0][0], a01 = dt * L[0][1], a10 = dt * L[1][0], a11 = dt * L[1][1];
        dD = (a00 + a11) + (a00 * a11 - a01 * a10);
    }
    dJ = dJ + dD + dJ * dD;
    T J = T(1) + dJ;
    T p = P.k_over_gamma * expm1(-P.gamma * log1p(dJ));
    s_iso = -P.vol0 * J * p;
}

// Viscous fluid (Sec. 2.3 eq:stress_strain with the rate d = (L + L^T)/2 in
// place of the printed increment): the Tait pressure of fluid_update plus
// 2 mu (d - tr(d)/D I), both at the updated J; S = V0 J' sigma, stored
// symmetric.
template <class T, int D>
__device__ __forceinline__ void vfluid_update(const Phys<T>& P, const T L[D][D], T& dJ, T S[D * (D + 1) / 2])
{
    T s_iso;
    fluid_update<T, D>(P, L, dJ, s_iso);
    T trd = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) trd += L[a][a];
    const T c = T(2) * P.visc * P.vol0 * (T(1) + dJ);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            T r = T(0.5) * (L[i][j] + L[j][i]);
            if (i == j) r -= trd / T(D);
            S[q] = c * r + ((i == j) ? s_iso : T(0));
        }
}

// Hypoelastic Drucker-Prager with the Jaumann rate and a tension cutoff
// (Sec. 2.3 eq:dp_stress; App. A).  The carried stress is S = V0 J sigma;
// the step's Cauchy stress is S / (V0 J) with J before its update
// J' = J det(I + dt L), and the new S is V0 J' sigma'.
//   trial = sigma + sigma Dw^T + Dw sigma^T + lam tr(Dd) I + 2 G Dd,
//     Dd = dt (L + L^T)/2, Dw = dt (L - L^T)/2
//   sigma_m = tr/D, s = trial - sigma_m I, tau = sqrt(s:s / 2)
//   f^s = tau - k_phi + q_phi sigma_m, f^t = sigma_m - sigma^t,
//   h = tau - tau^P - alpha^P (sigma_m - sigma^t)
//   zone I  (f^t < 0, f^s <= 0; or a trial of norm at the elastic band)
//   zone II (f^t < 0, f^s > 0; or f^t >= 0, h > 0): dl = f^s / (G + K q_phi q_psi),
//           sigma_m' = sigma_m - K q_psi dl, tau' = k_phi - q_phi sigma_m', s
//           scaled to tau'; a return beyond the cutoff ends at (sigma^t, tau^P)
//   zone III (f^t >= 0, h <= 0): sigma_m' = sigma^t, s kept
// de (optional) receives App. A's equivalent plastic strain increment:
// zone II dl sqrt(1/3 + 2/9 q_psi^2), zone III sqrt(2)/3 (sigma_m -
// sigma^t)/K, zone I 0.
template <class T, int D>
__device__ __forceinline__ void jaumann_update(const Phys<T>& P, const T L[D][D], T& dJ, T S[D * (D + 1) / 2],
                                               T* de = nullptr)
{
    constexpr int NS = D * (D + 1) / 2;
    const T Jo = T(1) + dJ;
    T s_unused;
    fluid_update<T, D>(P, L, dJ, s_unused);   // J' = J det(I + dt L) (its pressure is not used)
    const T Jn = T(1) + dJ;
    const T to_cauchy = T(1) / (P.vol0 * Jo);
    T sg[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            sg[i][j] = S[q] * to_cauchy;
            sg[j][i] = sg[i][j];
        }
    T Dd[D][D], Dw[D][D], trD = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            Dd[i][j] = T(0.5) * P.dt * (L[i][j] + L[j][i]);
            Dw[i][j] = T(0.5) * P.dt * (L[i][j] - L[j][i]);
        }
#pragma unroll
    for (int i = 0; i < D; ++i) trD += Dd[i][i];
    T tr[NS], sm = T(0), nrm2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            T r = sg[i][j];
#pragma unroll
            for (int k = 0; k < D; ++k) r += sg[i][k] * Dw[j][k] + sg[j][k] * Dw[i][k];
            r += T(2) * P.mu * Dd[i][j] + ((i == j) ? P.lam * trD : T(0));
            tr[q] = r;
            nrm2 += (i == j ? T(1) : T(2)) * r * r;
        }
#pragma unroll
    for (int i = 0; i < D; ++i) sm += tr[i];
    sm /= T(D);
    T ss2 = T(0);
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        if (q < D) tr[q] -= sm;   // deviator in place
        ss2 += (q < D ? T(1) : T(2)) * tr[q] * tr[q];
    }
    const T tau = sqrt(T(0.5) * ss2);
    const T fs = tau - P.jk_phi + P.jq_phi * sm;
    const T ft = sm - P.jst;
    const T hh = tau - P.jtauP - P.jalphaP * (sm - P.jst);
    int zone;
    if (nrm2 <= P.jband2) zone = 1;
    else if (ft < T(0)) zone = fs <= T(0) ? 1 : 2;
    else zone = hh > T(0) ? 2 : 3;
    T sm_n = sm, scale = T(1);
    if (de) *de = T(0);
    if (zone == 2) {
        const T dl = fs / (P.mu + P.jK * P.jq_phi * P.jq_psi);
        if (de) *de = dl * sqrt(T(1) / T(3) + T(2) / T(9) * P.jq_psi * P.jq_psi);
        sm_n = sm - P.jK * P.jq_psi * dl;
        T tau_n = P.jk_phi - P.jq_phi * sm_n;
        if (sm_n > P.jst) {
            sm_n = P.jst;
            tau_n = P.jtauP;
        }
        scale = tau > T(0) ? tau_n / tau : T(0);
    } else if (zone == 3) {
        if (de) *de = sqrt(T(2)) / T(3) * (sm - P.jst) / P.jK;
        sm_n = P.jst;
    }
    const T back = P.vol0 * Jn;
#pragma unroll
    for (int q = 0; q < NS; ++q) S[q] = back * (scale * tr[q] + ((q < D) ? sm_n : T(0)));
}

// Sand / elastic: F_tr = (I + dt L) F_e with F_e = I + G, so
// G_tr = G + dt (L + L G).  Hencky strain from b - I = G_tr + G_tr^T +
// G_tr G_tr^T: eps_i = log1p(eig_i)/2.  Return onto the Drucker-Prager cone:
//   apex (tr eps > 0)                 H = 0
//   elastic (dgamma <= 0)             H = eps
//   cone                              H = eps - dgamma dev/|dev|
// with dgamma = |dev| + (d lam + 2 mu)/(2 mu) alpha tr(eps).  Then
// F_e' = U diag(exp(H - eps)) U^T F_tr and tau = U diag(2 mu H + lam tr H) U^T.
template <class T, int D>
__device__ __forceinline__ bool hencky_eig(const Phys<T>& P, bool plastic, const T Gt[D][D], T G[D][D],
                                       T S[D * (D + 1) / 2], T* dgam = nullptr)
{
    bool conv = true;
    // b - I
    T B[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            T s = Gt[i][j] + Gt[j][i];
#pragma unroll
            for (int k = 0; k < D; ++k) s += Gt[i][k] * Gt[j][k];
            B[i][j] = s;
            B[j][i] = s;
        }
    T ev[D], U[D][D];
    if constexpr (D == 3) {
        T pk[6] = {B[0][0], B[1][1], B[2][2], B[0][1], B[0][2], B[1][2]};
        T V[3][3];
        conv = sym_eig3(pk, ev, V);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) U[i][j] = V[i][j];
    } else {
        T pk[3] = {B[0][0], B[1][1], B[0][1]};
        T V[2][2];
        sym_eig2(pk, ev, V);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) U[i][j] = V[i][j];
    }
    T eps[D], tr = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        eps[i] = T(0.5) * log1p(ev[i]);
        tr += eps[i];
    }
    T H[D];
    int cas = 1;   // 0 apex, 1 elastic, 2 cone
    T en2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) en2 += eps[i] * eps[i];
    if (dgam) *dgam = T(0);
    if (!plastic || en2 <= eps_elastic2<T>()) {
#pragma unroll
        for (int i = 0; i < D; ++i) H[i] = eps[i];
    } else if (tr > T(0)) {
        cas = 0;
        if (dgam) *dgam = sqrt(en2);
#pragma unroll
        for (int i = 0; i < D; ++i) H[i] = T(0);
    } else {
        T dev[D], dn2 = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            dev[i] = eps[i] - tr / T(D);
            dn2 += dev[i] * dev[i];
        }
        T dn = sqrt(dn2);
        T dg = dn + P.cone_coef * tr;
        if (dg <= T(0)) {
#pragma unroll
            for (int i = 0; i < D; ++i) H[i] = eps[i];
        } else {
            cas = 2;
            if (dgam) *dgam = dg;
            T r = dg / dn;
#pragma unroll
            for (int i = 0; i < D; ++i) H[i] = eps[i] - r * dev[i];
        }
    }
    T trH = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) trH += H[i];
    // stress
    T sig[D];
#pragma unroll
    for (int i = 0; i < D; ++i) sig[i] = P.vol0 * (T(2) * P.mu * H[i] + P.lam * trH);
    T Sf[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += U[i][k] * sig[k] * U[j][k];
            Sf[i][j] = s;
        }
    if constexpr (D == 3) {
        S[0] = Sf[0][0]; S[1] = Sf[1][1]; S[2] = Sf[2][2];
        S[3] = Sf[0][1]; S[4] = Sf[0][2]; S[5] = Sf[1][2];
    } else {
        S[0] = Sf[0][0]; S[1] = Sf[1][1]; S[2] = Sf[0][1];
    }
    if (cas == 1) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) G[i][j] = Gt[i][j];
        return conv;
    }
    // G' = U diag(expm1(H - eps)) U^T (I + G_tr) + G_tr
    T e1[D];
#pragma unroll
    for (int i = 0; i < D; ++i) e1[i] = expm1(H[i] - eps[i]);
    T M[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += U[i][k] * e1[k] * U[j][k];
            M[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = M[i][j];   // M * I
#pragma unroll
            for (int k = 0; k < D; ++k) s += M[i][k] * Gt[k][j];
            G[i][j] = Gt[i][j] + s;
        }
    return conv;
}

// Small symmetric matrices, packed: 3-D (xx,yy,zz,xy,xz,yz), 2-D (xx,yy,xy).
template <class T, int D> struct Sym;
template <class T> struct Sym<T, 3> {
    T a[6];
    __device__ __forceinline__ T tr() const { return a[0] + a[1] + a[2]; }
    __device__ __forceinline__ T norm2() const
    {
        return a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + T(2) * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]);
    }
    __device__ __forceinline__ T at(int i, int j) const
    {
        if (i == j) return a[i];
        int s = i + j;
        return a[s == 1 ? 3 : (s == 2 ? 4 : 5)];
    }
};
template <class T> struct Sym<T, 2> {
    T a[3];
    __device__ __forceinline__ T tr() const { return a[0] + a[1]; }
    __device__ __forceinline__ T norm2() const { return a[0] * a[0] + a[1] * a[1] + T(2) * a[2] * a[2]; }
    __device__ __forceinline__ T at(int i, int j) const { return i == j ? a[i] : a[2]; }
};

// c I + A B for commuting symmetric A, B (the product is symmetric)
template <class T>
__device__ __forceinline__ Sym<T, 3> cI_plus_AB(T c, const Sym<T, 3>& A, const Sym<T, 3>& B)
{
    Sym<T, 3> R;
    R.a[0] = c + A.a[0] * B.a[0] + A.a[3] * B.a[3] + A.a[4] * B.a[4];
    R.a[1] = c + A.a[3] * B.a[3] + A.a[1] * B.a[1] + A.a[5] * B.a[5];
    R.a[2] = c + A.a[4] * B.a[4] + A.a[5] * B.a[5] + A.a[2] * B.a[2];
    R.a[3] = A.a[0] * B.a[3] + A.a[3] * B.a[1] + A.a[4] * B.a[5];
    R.a[4] = A.a[0] * B.a[4] + A.a[3] * B.a[5] + A.a[4] * B.a[2];
    R.a[5] = A.a[3] * B.a[4] + A.a[1] * B.a[5] + A.a[5] * B.a[2];
    return R;
}
template <class T>
__device__ __forceinline__ Sym<T, 2> cI_plus_AB(T c, const Sym<T, 2>& A, const Sym<T, 2>& B)
{
    Sym<T, 2> R;
    R.a[0] = c + A.a[0] * B.a[0] + A.a[2] * B.a[2];
    R.a[1] = c + A.a[2] * B.a[2] + A.a[1] * B.a[1];
    R.a[2] = A.a[0] * B.a[2] + A.a[2] * B.a[1];
    return R;
}

// Truncated series for the matrix functions of a small symmetric argument:
// log(I + X) = sum_k (-1)^(k+1) X^k / k and exp(Y) - I = sum_k Y^k / k!, by
// Horner's rule.  Used when |X|_F, |Y|_F < kMax: the first omitted term,
// relative to the result, is then at or below the unit roundoff (float:
// 0.02^4/5 = 3.2e-8 for log with kLog = 4, 0.02^4/5! = 1.3e-9 for exp;
// double: 0.01^9/10 = 1e-19 and 0.01^7/8! = 2.5e-19).
template <class T> struct Series;
template <> struct Series<float> { static constexpr float kMax = 0.02f; static constexpr int kLog = 4, kExp = 4; };
template <> struct Series<double> { static constexpr double kMax = 0.01; static constexpr int kLog = 9, kExp = 7; };

template <class T, int D>
__device__ __forceinline__ Sym<T, D> log1p_sym(const Sym<T, D>& X)
{
    constexpr int K = Series<T>::kLog;
    Sym<T, D> Pm;
    T cK = ((K & 1) ? T(1) : T(-1)) / T(K);
#pragma unroll
    for (int q = 0; q < (D == 3 ? 6 : 3); ++q) Pm.a[q] = (q < D) ? cK : T(0);
#pragma unroll
    for (int k = K - 1; k >= 1; --k) Pm = cI_plus_AB(((k & 1) ? T(1) : T(-1)) / T(k), X, Pm);
    return cI_plus_AB(T(0), X, Pm);
}

template <class T, int D>
__device__ __forceinline__ Sym<T, D> expm1_sym(const Sym<T, D>& Y)
{
    constexpr int K = Series<T>::kExp;
    Sym<T, D> Pm;
#pragma unroll
    for (int q = 0; q < (D == 3 ? 6 : 3); ++q) Pm.a[q] = (q < D) ? T(1) : T(0);
#pragma unroll
    for (int k = K; k >= 2; --k) {
        Sym<T, D> Z = Y;
#pragma unroll
        for (int q = 0; q < (D == 3 ? 6 : 3); ++q) Z.a[q] *= T(1) / T(k);
        Pm = cI_plus_AB(T(1), Z, Pm);
    }
    return cI_plus_AB(T(0), Y, Pm);
}

// Hencky return written on the strain tensor E = log(b)/2 itself: every
// quantity of the return (trace, deviator, its norm, the projected H, the
// stress) is a polynomial in E, so no eigenvectors are needed while
// b - I and the correction exp(H - E) are small enough for the series.
// Returns false when they are not (the caller then takes hencky_eig).
template <class T, int D>
__device__ __forceinline__ bool hencky_series(const Phys<T>& P, bool plastic, const T Gt[D][D], T G[D][D],
                                              T S[D * (D + 1) / 2], T* dgam = nullptr)
{
    constexpr int NS = D * (D + 1) / 2;
    Sym<T, D> X;   // b - I = Gt + Gt^T + Gt Gt^T
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            T s = Gt[i][j] + Gt[j][i];
#pragma unroll
            for (int k = 0; k < D; ++k) s += Gt[i][k] * Gt[j][k];
            int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            X.a[q] = s;
        }
    const T lim2 = Series<T>::kMax * Series<T>::kMax;
    if (!(X.norm2() < lim2)) return false;
    Sym<T, D> E = log1p_sym(X);
#pragma unroll
    for (int q = 0; q < NS; ++q) E.a[q] *= T(0.5);
    T trE = E.tr();
    Sym<T, D> Eh = E;
#pragma unroll
    for (int i = 0; i < D; ++i) Eh.a[i] -= trE * (T(1) / T(D));
    T n = sqrt(Eh.norm2());
    int cas = 1;
    T r = T(0);   // H = E - r * Ehat (cone), 0 (apex), E (elastic)
    T dgv = T(0);
    if (plastic && E.norm2() > eps_elastic2<T>()) {
        if (trE > T(0)) {
            cas = 0;
            dgv = sqrt(E.norm2());
        } else {
            T dg = n + P.cone_coef * trE;
            if (dg > T(0)) {
                cas = 2;
                r = dg / n;
                dgv = dg;
            }
        }
    }
    Sym<T, D> Y;   // H - E
    if (cas == 0) {
#pragma unroll
        for (int q = 0; q < NS; ++q) Y.a[q] = -E.a[q];
    } else if (cas == 2) {
#pragma unroll
        for (int q = 0; q < NS; ++q) Y.a[q] = -r * Eh.a[q];
    }
    if (cas != 1 && !(Y.norm2() < lim2)) return false;
    if (dgam) *dgam = dgv;
    // stress: tau = 2 mu H + lam tr(H) I
    T trH = (cas == 0) ? T(0) : trE;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        T h = (cas == 0) ? T(0) : (cas == 2 ? E.a[q] - r * Eh.a[q] : E.a[q]);
        S[q] = P.vol0 * (T(2) * P.mu * h + ((q < D) ? P.lam * trH : T(0)));
    }
    if (cas == 1) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) G[i][j] = Gt[i][j];
        return true;
    }
    // F_e' = exp(Y) F_tr:  G' = (exp(Y) - I)(I + Gt) + Gt
    Sym<T, D> M = expm1_sym(Y);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = M.at(i, j);
#pragma unroll
            for (int k = 0; k < D; ++k) s += M.at(i, k) * Gt[k][j];
            G[i][j] = Gt[i][j] + s;
        }
    return true;
}

// Returns false when the binary64 eigen-solve of the fallback did not
// converge within its sweep budget (the caller latches it).
template <class T, int D>
__device__ __forceinline__ bool hencky_update(const Phys<T>& P, bool plastic, const T L[D][D],
                                              T G[D][D], T S[D * (D + 1) / 2], T* dgam = nullptr)
{
    T dt = P.dt;
    T Gt[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T lg = L[i][j];
#pragma unroll
            for (int k = 0; k < D; ++k) lg += L[i][k] * G[k][j];
            Gt[i][j] = G[i][j] + dt * lg;
        }
    if (hencky_series<T, D>(P, plastic, Gt, G, S, dgam)) return true;
    return hencky_eig<T, D>(P, plastic, Gt, G, S, dgam);
}

// ---------------------------------------------------------------------------
// Walls (Sec. 2.2 ghost cells; Sec. 5.3 Coulomb law at a resting wall).
// ---------------------------------------------------------------------------

template <class T, int D>
__device__ __forceinline__ void wall_node(int mode, T mu, int axis, T sign, T v[D])
{
    T vn = sign * v[axis];
    if (!(vn > T(0))) return;
    if (mode == WALL_STICK) {
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] = T(0);
        return;
    }
    v[axis] = T(0);   // tangential part left
    if (mode == WALL_SLIP) return;
    T vt2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) vt2 += v[a] * v[a];
    T vt = sqrt(vt2);
    if (vt <= mu * vn) {
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] = T(0);
    } else {
        T sc = T(1) - mu * vn / vt;
#pragma unroll
        for (int a = 0; a < D; ++a) v[a] *= sc;
    }
}

// Resting rigid boxes (Sec. 4.2.1, frictionless contact): a node with mass
// inside the closed box loses the velocity component that points into the
// box through its nearest face (faces on the domain boundary excluded; ties
// to the first face in the order x-, x+, y-, y+, z-, z+).  xi: the node's
// position.  obstacle_component returns the axis of the component that
// obstacle o removes from a node moving with v, or -1.
template <class T, int D>
__device__ __forceinline__ int obstacle_component(const Phys<T>& P, int o, const double xi[D], const T v[D])
{
    bool inside = true;
#pragma unroll
    for (int a = 0; a < D; ++a) inside &= xi[a] >= P.obst_lo[o][a] && xi[a] <= P.obst_hi[o][a];
    if (!inside) return -1;
    int best = -1;
    double bd = 0.0;
#pragma unroll
    for (int f = 0; f < 2 * D; ++f) {
        if (!((P.obst_face_ok[o] >> f) & 1)) continue;
        const int a = f >> 1;
        const double depth = (f & 1) ? P.obst_hi[o][a] - xi[a] : xi[a] - P.obst_lo[o][a];
        if (best < 0 || depth < bd) {
            best = f;
            bd = depth;
        }
    }
    if (best < 0) return -1;
    const int a = best >> 1;
    // the normal points into the obstacle: +e_a through its lower face
    const T vn = (best & 1) ? -v[a] : v[a];
    return vn > T(0) ? a : -1;
}

template <class T, int D>
__device__ __forceinline__ void obstacle_node(const Phys<T>& P, const double xi[D], T v[D])
{
    for (int o = 0; o < P.n_obst; ++o) {
        const int a = obstacle_component<T, D>(P, o, xi, v);
        if (a >= 0) v[a] = T(0);
    }
}

}  // namespace mpm
