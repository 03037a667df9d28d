// Device-side vector-Jacobian products of the constitutive updates and the
// walls: the reverse of hencky_update, fluid_update and wall_node.
//
// The Hencky map is an isotropic function of b = F_tr F_tr^T: with
// b = U diag(1 + beta) U^T every intermediate (E = log(b)/2, its deviator,
// exp of the return) shares the eigenbasis U, and the derivative of a matrix
// function f in that basis multiplies component (i,j) by the divided
// difference f[l_i, l_j] (f'(l_i) on the diagonal).  Repeated eigenvalues
// (F = I at rest) take the limit, evaluated by series.
#pragma once

#include "mpm_device.hpp"

namespace mpm {

template <class T> struct SeriesTol;
template <> struct SeriesTol<float> { static constexpr float dl = 1e-3f, de = 1e-3f; };
template <> struct SeriesTol<double> { static constexpr double dl = 1e-5, de = 1e-6; };

// [f(bi) - f(bj)] / (bi - bj) for f(b) = log1p(b)/2
template <class T>
__device__ __forceinline__ T dd_halflog1p(T bi, T bj)
{
    T inv = T(1) / (T(1) + bj);
    T del = (bi - bj) * inv;
    if (fabs(del) < SeriesTol<T>::dl) return T(0.5) * inv * (T(1) - del * (T(0.5) - del * (T(1) / T(3))));
    return T(0.5) * log1p(del) / (bi - bj);
}

// [exp(yi) - exp(yj)] / (yi - yj)
template <class T>
__device__ __forceinline__ T dd_exp(T yi, T yj)
{
    T del = yi - yj;
    if (fabs(del) < SeriesTol<T>::de) return exp(yj) * (T(1) + del * (T(0.5) + del * (T(1) / T(6))));
    return exp(yj) * expm1(del) / del;
}

template <class T, int D>
__device__ __forceinline__ void to_eig(const T U[D][D], const T A[D][D], T R[D][D])   // R = U^T A U
{
    T tmp[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += A[i][k] * U[k][j];
            tmp[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += U[k][i] * tmp[k][j];
            R[i][j] = s;
        }
}

template <class T, int D>
__device__ __forceinline__ void from_eig(const T U[D][D], const T A[D][D], T R[D][D])   // R = U A U^T
{
    T tmp[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += A[i][k] * U[j][k];
            tmp[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += U[i][k] * tmp[k][j];
            R[i][j] = s;
        }
}

// Reverse of hencky_update through the eigen-decomposition of b (any
// strain).  Inputs: the velocity gradient L and stored G = F_e - I of the
// step, the adjoints of the outputs (Gb_out for F_e', sb_out for the stored
// symmetric stress).  Outputs: Lb and Gb_in.
template <class T, int D>
__device__ __forceinline__ void hencky_vjp_eig(const Phys<T>& P, bool plastic, const T L[D][D], const T G[D][D],
                                               const T Gb_out[D][D], const T sb_out[D * (D + 1) / 2], T Lb[D][D],
                                               T Gb_in[D][D])
{
    const T dt = P.dt;
    T Gt[D][D], Ft[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T lg = L[i][j];
#pragma unroll
            for (int k = 0; k < D; ++k) lg += L[i][k] * G[k][j];
            Gt[i][j] = G[i][j] + dt * lg;
            Ft[i][j] = Gt[i][j] + ((i == j) ? T(1) : T(0));
        }
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
    T beta[D], U[D][D];
    if constexpr (D == 3) {
        T pk[6] = {B[0][0], B[1][1], B[2][2], B[0][1], B[0][2], B[1][2]};
        T V[3][3];
        sym_eig3(pk, beta, V);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) U[i][j] = V[i][j];
    } else {
        T pk[3] = {B[0][0], B[1][1], B[0][1]};
        T V[2][2];
        sym_eig2(pk, beta, V);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) U[i][j] = V[i][j];
    }
    T eps[D], tr = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        eps[i] = T(0.5) * log1p(beta[i]);
        tr += eps[i];
    }
    T dev[D], dn2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        dev[i] = eps[i] - tr / T(D);
        dn2 += dev[i] * dev[i];
    }
    T dn = sqrt(dn2);
    int cas = 1;
    T en2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) en2 += eps[i] * eps[i];
    if (plastic && en2 > eps_elastic2<T>()) {
        if (tr > T(0)) cas = 0;
        else if (dn + P.cone_coef * tr > T(0)) cas = 2;
    }
    // adjoint of the symmetric stress, scaled by V0 (S = V0 tau)
    T taub[D][D];
    if constexpr (D == 3) {
        taub[0][0] = sb_out[0]; taub[1][1] = sb_out[1]; taub[2][2] = sb_out[2];
        taub[0][1] = taub[1][0] = T(0.5) * sb_out[3];
        taub[0][2] = taub[2][0] = T(0.5) * sb_out[4];
        taub[1][2] = taub[2][1] = T(0.5) * sb_out[5];
    } else {
        taub[0][0] = sb_out[0]; taub[1][1] = sb_out[1];
        taub[0][1] = taub[1][0] = T(0.5) * sb_out[2];
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) taub[i][j] *= P.vol0;
    T Tt[D][D];
    to_eig<T, D>(U, taub, Tt);
    T trT = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) trT += Tt[i][i];

    T Ftb[D][D], Et[D][D];
    if (cas == 1) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                Ftb[i][j] = Gb_out[i][j];
                Et[i][j] = T(2) * P.mu * Tt[i][j] + ((i == j) ? P.lam * trT : T(0));
            }
    } else {
        T kappa = (cas == 2) ? T(1) + P.cone_coef * tr / dn : T(0);
        T y[D], ey[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            y[i] = (cas == 0) ? -eps[i] : -kappa * dev[i];
            ey[i] = exp(y[i]);
        }
        // X = U diag(exp y) U^T ; F_e' = X F_tr
        T X[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T s = T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) s += U[i][k] * ey[k] * U[j][k];
                X[i][j] = s;
            }
        T Xb[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T f = T(0), xb = T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    f += X[i][k] * Gb_out[k][j];          // X symmetric: X^T Gb
                    xb += Gb_out[i][k] * Ft[j][k];        // Gb F_tr^T
                }
                Ftb[i][j] = f;
                Xb[i][j] = xb;
            }
        T Xs[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Xs[i][j] = T(0.5) * (Xb[i][j] + Xb[j][i]);
        T Xt[D][D], Yt[D][D];
        to_eig<T, D>(U, Xs, Xt);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Yt[i][j] = Xt[i][j] * ((i == j) ? ey[i] : dd_exp(y[i], y[j]));
        if (cas == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) Et[i][j] = -Yt[i][j];
        } else {
            const T a1 = T(2) * P.mu / T(D) + P.lam, b1 = T(2) * P.mu * P.cone_coef, c = P.cone_coef;
            T Eht[D][D];
            T kb = T(0), sTd = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                kb -= Yt[i][i] * dev[i];
                sTd += Tt[i][i] * dev[i];
            }
            // ratios first: tr/dn is bounded on the cone, dn^2 may underflow
            const T td = tr / dn;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) Eht[i][j] = -kappa * Yt[i][j] - b1 * td * Tt[i][j];
            T trb = a1 * trT - b1 * sTd / dn + kb * c / dn;
            T nb = (b1 * td * sTd - kb * c * td) / dn;
#pragma unroll
            for (int i = 0; i < D; ++i) Eht[i][i] += nb * (dev[i] / dn);
            T trE = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) trE += Eht[i][i];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) Et[i][j] = Eht[i][j] + ((i == j) ? trb - trE / T(D) : T(0));
        }
    }
    // E = log1p(b - I)/2 : b bar in the eigenbasis, then back
    T bt[D][D], bb[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j)
            bt[i][j] = Et[i][j] * ((i == j) ? T(0.5) / (T(1) + beta[i]) : dd_halflog1p(beta[i], beta[j]));
    from_eig<T, D>(U, bt, bb);
    // b = F_tr F_tr^T
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += (bb[i][k] + bb[k][i]) * Ft[k][j];
            Ftb[i][j] += s;
        }
    // F_tr = (I + dt L) F
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T l = T(0), g = Ftb[i][j];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                l += Ftb[i][k] * (G[j][k] + ((j == k) ? T(1) : T(0)));
                g += dt * L[k][i] * Ftb[k][j];
            }
            Lb[i][j] = dt * l;
            Gb_in[i][j] = g;
        }
}

// General D x D matrix (the adjoints are not symmetric in general).
template <class T, int D> struct Gen {
    T a[D][D];
};

template <class T, int D>
__device__ __forceinline__ Gen<T, D> sym_gen(const Sym<T, D>& X, const Gen<T, D>& A)   // X A
{
    Gen<T, D> R;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += X.at(i, k) * A.a[k][j];
            R.a[i][j] = s;
        }
    return R;
}

template <class T, int D>
__device__ __forceinline__ Gen<T, D> gen_sym(const Gen<T, D>& A, const Sym<T, D>& X)   // A X
{
    Gen<T, D> R;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) s += A.a[i][k] * X.at(k, j);
            R.a[i][j] = s;
        }
    return R;
}

template <class T, int D>
__device__ __forceinline__ Sym<T, D> sym_part(const Gen<T, D>& A, T scale)   // scale (A + A^T) / 2
{
    Sym<T, D> R;
#pragma unroll
    for (int i = 0; i < D; ++i) R.a[i] = scale * A.a[i][i];
    if constexpr (D == 3) {
        R.a[3] = T(0.5) * scale * (A.a[0][1] + A.a[1][0]);
        R.a[4] = T(0.5) * scale * (A.a[0][2] + A.a[2][0]);
        R.a[5] = T(0.5) * scale * (A.a[1][2] + A.a[2][1]);
    } else {
        R.a[2] = T(0.5) * scale * (A.a[0][1] + A.a[1][0]);
    }
    return R;
}

// Frechet derivatives of the truncated series of hencky_series, applied to
// a direction A: D f(X)[A] = sum_k c_k sum_{j<k} X^j A X^(k-1-j).  For
// symmetric X this map is its own adjoint in the Frobenius product, so it
// is also the vector-Jacobian product.  Evaluated by carrying the derivative
// through the same Horner recurrence (the upper-right block of f applied to
// [[X, A], [0, X]]).
template <class T, int D>
__device__ __forceinline__ Gen<T, D> dlog1p_sym(const Sym<T, D>& X, const Gen<T, D>& A)
{
    constexpr int K = Series<T>::kLog;
    constexpr int NS = D * (D + 1) / 2;
    Sym<T, D> P1;
    Gen<T, D> P2;
    T cK = ((K & 1) ? T(1) : T(-1)) / T(K);
#pragma unroll
    for (int q = 0; q < NS; ++q) P1.a[q] = (q < D) ? cK : T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) P2.a[i][j] = T(0);
#pragma unroll
    for (int k = K - 1; k >= 1; --k) {
        Gen<T, D> t1 = sym_gen(X, P2), t2 = gen_sym(A, P1);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) P2.a[i][j] = t1.a[i][j] + t2.a[i][j];
        P1 = cI_plus_AB(((k & 1) ? T(1) : T(-1)) / T(k), X, P1);
    }
    Gen<T, D> t1 = sym_gen(X, P2), t2 = gen_sym(A, P1);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) t1.a[i][j] += t2.a[i][j];
    return t1;
}

template <class T, int D>
__device__ __forceinline__ Gen<T, D> dexpm1_sym(const Sym<T, D>& Y, const Gen<T, D>& A)
{
    constexpr int K = Series<T>::kExp;
    constexpr int NS = D * (D + 1) / 2;
    Sym<T, D> P1;
    Gen<T, D> P2;
#pragma unroll
    for (int q = 0; q < NS; ++q) P1.a[q] = (q < D) ? T(1) : T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) P2.a[i][j] = T(0);
#pragma unroll
    for (int k = K; k >= 2; --k) {
        const T ik = T(1) / T(k);
        Gen<T, D> t1 = sym_gen(Y, P2), t2 = gen_sym(A, P1);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) P2.a[i][j] = ik * (t1.a[i][j] + t2.a[i][j]);
        Sym<T, D> Z = Y;
#pragma unroll
        for (int q = 0; q < NS; ++q) Z.a[q] *= ik;
        P1 = cI_plus_AB(T(1), Z, P1);
    }
    Gen<T, D> t1 = sym_gen(Y, P2), t2 = gen_sym(A, P1);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) t1.a[i][j] += t2.a[i][j];
    return t1;
}

// Reverse of the series form of the Hencky return (hencky_series), valid
// where that form was taken; returns false otherwise (then the caller takes
// hencky_vjp_eig).  With Hb the adjoint of H from the stress and Gb_out that
// of F_e' = exp(Y) F_tr (Y = H - E):
//   F_tr bar = Gb_out + (exp(Y) - I) Gb_out,   exp(Y) bar = Gb_out F_tr^T,
//   Y bar = D expm1(Y)[exp(Y) bar],
//   E bar = Hb (elastic), -Y bar (apex), or, on the cone (Y = -r dev E,
//   r = 1 + c tr E / |dev E|):  Hb + dev(W) - (c z / n) I with Z = Hb + Y bar,
//   z = <Z, dev E>, n = |dev E|, W = (c z tr E / n^3) dev E - r Z;
//   X bar = D log1p(X)[E bar] / 2,  F_tr bar += 2 X bar F_tr.
template <class T, int D>
__device__ __forceinline__ bool hencky_vjp_series(const Phys<T>& P, bool plastic, const T L[D][D], const T G[D][D],
                                                  const T Gb_out[D][D], const T sb_out[D * (D + 1) / 2],
                                                  T Lb[D][D], T Gb_in[D][D])
{
    constexpr int NS = D * (D + 1) / 2;
    const T dt = P.dt;
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
    // forward, as hencky_series
    Sym<T, D> X;
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
    for (int i = 0; i < D; ++i) Eh.a[i] -= trE / T(D);
    T n = sqrt(Eh.norm2());
    int cas = 1;
    T r = T(0);
    if (plastic && E.norm2() > eps_elastic2<T>()) {
        if (trE > T(0)) cas = 0;
        else {
            T dg = n + P.cone_coef * trE;
            if (dg > T(0)) {
                cas = 2;
                r = dg / n;
            }
        }
    }
    Sym<T, D> Y;
    if (cas == 0) {
#pragma unroll
        for (int q = 0; q < NS; ++q) Y.a[q] = -E.a[q];
    } else {
#pragma unroll
        for (int q = 0; q < NS; ++q) Y.a[q] = -r * Eh.a[q];
    }
    if (cas != 1 && !(Y.norm2() < lim2)) return false;
    // adjoint of H from the stored stress S = V0 (2 mu H + lam tr(H) I)
    Sym<T, D> tb;
#pragma unroll
    for (int q = 0; q < NS; ++q) tb.a[q] = P.vol0 * ((q < D) ? sb_out[q] : T(0.5) * sb_out[q]);
    T trt = tb.tr();
    Sym<T, D> Hb;
#pragma unroll
    for (int q = 0; q < NS; ++q) Hb.a[q] = T(2) * P.mu * tb.a[q] + ((q < D) ? P.lam * trt : T(0));
    Gen<T, D> Ftb;   // adjoint of F_tr (equivalently of G_tr)
    Sym<T, D> Eb;
    if (cas == 1) {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Ftb.a[i][j] = Gb_out[i][j];
        Eb = Hb;
    } else {
        Sym<T, D> M = expm1_sym(Y);
        Gen<T, D> Mb;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T f = Gb_out[i][j], mb = Gb_out[i][j];   // F_tr^T = I + Gt^T
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    f += M.at(i, k) * Gb_out[k][j];
                    mb += Gb_out[i][k] * Gt[j][k];
                }
                Ftb.a[i][j] = f;
                Mb.a[i][j] = mb;
            }
        Sym<T, D> Yb = sym_part(dexpm1_sym(Y, Mb), T(1));
        if (cas == 0) {
#pragma unroll
            for (int q = 0; q < NS; ++q) Eb.a[q] = -Yb.a[q];
        } else {
            const T c = P.cone_coef;
            Sym<T, D> Z;
#pragma unroll
            for (int q = 0; q < NS; ++q) Z.a[q] = Hb.a[q] + Yb.a[q];
            // <Z, dev E> in the full-matrix Frobenius product, divided by
            // n; the factors are formed so that nothing underflows when the
            // strain is tiny (n^3 would)
            T z = T(0);
#pragma unroll
            for (int q = 0; q < NS; ++q) z += ((q < D) ? T(1) : T(2)) * Z.a[q] * Eh.a[q];
            const T zn = z / n, tn = trE / n;
            const T cw = c * zn * tn / n;
            Sym<T, D> Wm;
#pragma unroll
            for (int q = 0; q < NS; ++q) Wm.a[q] = cw * Eh.a[q] - r * Z.a[q];
            T trW = Wm.tr();
#pragma unroll
            for (int q = 0; q < NS; ++q)
                Eb.a[q] = Hb.a[q] + Wm.a[q] + ((q < D) ? -trW / T(D) - c * zn : T(0));
        }
    }
    // E = log1p(X) / 2
    Gen<T, D> Ebg;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) Ebg.a[i][j] = Eb.at(i, j);
    Sym<T, D> Xb = sym_part(dlog1p_sym(X, Ebg), T(0.5));
    // X = Gt + Gt^T + Gt Gt^T:  Gt bar += 2 Xb (I + Gt)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T s = Xb.at(i, j);
#pragma unroll
            for (int k = 0; k < D; ++k) s += Xb.at(i, k) * Gt[k][j];
            Ftb.a[i][j] += T(2) * s;
        }
    // Gt = G + dt L (I + G)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T l = T(0), g = Ftb.a[i][j];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                l += Ftb.a[i][k] * (G[j][k] + ((j == k) ? T(1) : T(0)));
                g += dt * L[k][i] * Ftb.a[k][j];
            }
            Lb[i][j] = dt * l;
            Gb_in[i][j] = g;
        }
    return true;
}

// Reverse of hencky_update: the series form where the forward took it, the
// eigen form otherwise.
template <class T, int D>
__device__ __forceinline__ void hencky_vjp(const Phys<T>& P, bool plastic, const T L[D][D], const T G[D][D],
                                           const T Gb_out[D][D], const T sb_out[D * (D + 1) / 2], T Lb[D][D],
                                           T Gb_in[D][D])
{
    if (!hencky_vjp_series<T, D>(P, plastic, L, G, Gb_out, sb_out, Lb, Gb_in))
        hencky_vjp_eig<T, D>(P, plastic, L, G, Gb_out, sb_out, Lb, Gb_in);
}

// Reverse of jaumann_update (hypoelastic Drucker-Prager, App. A) with the
// zone held fixed.  Inputs: the step's velocity gradient L, the stored
// J - 1 and stress cache S (packed symmetric, V0 J sigma), and the adjoints
// Jb_out, Sb_out of the outputs J' - 1 and S'.  Outputs: Lb, and the
// adjoints Jb_in, Sb_in of the inputs.  Written on full matrices: a packed
// off-diagonal value stands for two entries, so its adjoint is the sum of
// theirs.
template <class T, int D>
__device__ __forceinline__ void jaumann_vjp(const Phys<T>& P, const T L[D][D], T dJ, const T S[D * (D + 1) / 2],
                                            T Jb_out, const T Sb_out[D * (D + 1) / 2], T Lb[D][D], T& Jb_in,
                                            T Sb_in[D * (D + 1) / 2])
{
    constexpr int NS = D * (D + 1) / 2;
    const T dt = P.dt;
    // ---- forward, keeping what the reverse needs
    T M[D][D], cof[D][D], detM;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) M[i][j] = ((i == j) ? T(1) : T(0)) + dt * L[i][j];
    if constexpr (D == 3) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                cof[i][j] = M[i1][j1] * M[i2][j2] - M[i1][j2] * M[i2][j1];
            }
        detM = M[0][0] * cof[0][0] + M[0][1] * cof[0][1] + M[0][2] * cof[0][2];
    } else {
        cof[0][0] = M[1][1]; cof[0][1] = -M[1][0];
        cof[1][0] = -M[0][1]; cof[1][1] = M[0][0];
        detM = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    }
    const T Jo = T(1) + dJ;
    const T Jn = Jo * detM;
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
            Dd[i][j] = T(0.5) * dt * (L[i][j] + L[j][i]);
            Dw[i][j] = T(0.5) * dt * (L[i][j] - L[j][i]);
        }
#pragma unroll
    for (int i = 0; i < D; ++i) trD += Dd[i][i];
    T sv[D][D], sm = T(0), nrm2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T r = sg[i][j];
#pragma unroll
            for (int k = 0; k < D; ++k) r += sg[i][k] * Dw[j][k] + sg[j][k] * Dw[i][k];
            r += T(2) * P.mu * Dd[i][j] + ((i == j) ? P.lam * trD : T(0));
            sv[i][j] = r;
            nrm2 += r * r;
        }
#pragma unroll
    for (int i = 0; i < D; ++i) sm += sv[i][i];
    sm /= T(D);
    T ss2 = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        sv[i][i] -= sm;
#pragma unroll
        for (int j = 0; j < D; ++j) ss2 += sv[i][j] * sv[i][j];
    }
    const T tau = sqrt(T(0.5) * ss2);
    const T fs = tau - P.jk_phi + P.jq_phi * sm;
    const T ft = sm - P.jst;
    const T hh = tau - P.jtauP - P.jalphaP * (sm - P.jst);
    int zone;
    if (nrm2 <= P.jband2) zone = 1;
    else if (ft < T(0)) zone = fs <= T(0) ? 1 : 2;
    else zone = hh > T(0) ? 2 : 3;
    const T den = P.mu + P.jK * P.jq_phi * P.jq_psi;
    T sm_n = sm, scale = T(1), tau_n = T(0);
    bool corner = false;
    if (zone == 2) {
        sm_n = sm - P.jK * P.jq_psi * fs / den;
        tau_n = P.jk_phi - P.jq_phi * sm_n;
        if (sm_n > P.jst) {
            corner = true;
            sm_n = P.jst;
            tau_n = P.jtauP;
        }
        scale = tau > T(0) ? tau_n / tau : T(0);
    } else if (zone == 3) {
        sm_n = P.jst;
    }
    // ---- reverse
    // S'_q = V0 J' sigma'_q, J' = Jn
    T Jnb = Jb_out;
    T SgB[D][D];   // full-matrix adjoint of sigma'
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            const T so = scale * sv[i][j] + ((i == j) ? sm_n : T(0));
            Jnb += P.vol0 * Sb_out[q] * so;
            const T b = P.vol0 * Jn * Sb_out[q] * ((i == j) ? T(1) : T(0.5));
            SgB[i][j] = b;
            SgB[j][i] = b;
        }
    // sigma' = scale s + sm_n I
    T sB[D][D], scaleB = T(0), smnB = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        smnB += SgB[i][i];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            sB[i][j] = scale * SgB[i][j];
            scaleB += SgB[i][j] * sv[i][j];
        }
    }
    T smB = T(0), tauB = T(0);
    if (zone == 1) {
        smB += smnB;
    } else if (zone == 2) {
        // scale = tau_n / tau (0 and constant at tau = 0)
        const T taunB = tau > T(0) ? scaleB / tau : T(0);
        if (tau > T(0)) tauB += -scaleB * tau_n / (tau * tau);
        if (!corner) {
            const T smnB2 = smnB - P.jq_phi * taunB;   // tau_n = k_phi - q_phi sm_n
            smB += smnB2;
            const T fsB = -P.jK * P.jq_psi / den * smnB2;
            tauB += fsB;
            smB += P.jq_phi * fsB;
        }
    }
    // tau = sqrt(s:s / 2), s = T - sm I, sm = tr(T)/D
    if (tau > T(0)) {
        const T c = tauB / (T(2) * tau);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) sB[i][j] += c * sv[i][j];
    }
    T trsB = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) trsB += sB[i][i];
    T TB[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) TB[i][j] = sB[i][j] + ((i == j) ? (smB - trsB) / T(D) : T(0));
    // T = sigma + sigma Dw^T + Dw sigma^T + 2 G Dd + lam tr(Dd) I
    T sgB[D][D], DwB[D][D], trTB = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) trTB += TB[i][i];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            T r = TB[a][b], w = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                r += TB[a][k] * Dw[k][b] + TB[k][a] * Dw[k][b];
                w += TB[k][a] * sg[k][b] + TB[a][k] * sg[k][b];
            }
            sgB[a][b] = r;
            DwB[a][b] = w;
        }
    // Dd = dt sym(L), Dw = dt skew(L); J' = J det(M) with M = I + dt L
    const T detB = Jnb * Jo;
    T JoB = Jnb * detM;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            const T DdB_ab = T(2) * P.mu * TB[a][b] + ((a == b) ? P.lam * trTB : T(0));
            const T DdB_ba = T(2) * P.mu * TB[b][a] + ((a == b) ? P.lam * trTB : T(0));
            Lb[a][b] = T(0.5) * dt * (DdB_ab + DdB_ba) + T(0.5) * dt * (DwB[a][b] - DwB[b][a]) + detB * dt * cof[a][b];
        }
    // sigma = S / (V0 J)
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            const T bq = (i == j) ? sgB[i][i] : sgB[i][j] + sgB[j][i];
            Sb_in[q] = bq * to_cauchy;
            JoB -= bq * sg[i][j] / Jo;
        }
    Jb_in = JoB;
    (void)NS;
}

// Reverse of fluid_update: Jb_out and sb_out are the adjoints of J' - 1 and
// of the isotropic stress value; dJ is the stored J - 1 of the step.
template <class T, int D>
__device__ __forceinline__ void fluid_vjp(const Phys<T>& P, const T L[D][D], T dJ, T Jb_out, T sb_out,
                                          T Lb[D][D], T& Jb_in)
{
    const T dt = P.dt;
    T M[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) M[i][j] = ((i == j) ? T(1) : T(0)) + dt * L[i][j];
    T cof[D][D], detM;
    if constexpr (D == 3) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                cof[i][j] = M[i1][j1] * M[i2][j2] - M[i1][j2] * M[i2][j1];
            }
        T A[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) A[i][j] = dt * L[i][j];
        T trA = A[0][0] + A[1][1] + A[2][2];
        T m2 = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) + (A[0][0] * A[2][2] - A[0][2] * A[2][0]) +
               (A[1][1] * A[2][2] - A[1][2] * A[2][1]);
        T det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        detM = T(1) + (trA + m2 + det);
    } else {
        cof[0][0] = M[1][1]; cof[0][1] = -M[1][0];
        cof[1][0] = -M[0][1]; cof[1][1] = M[0][0];
        T a00 = dt * L[0][0], a01 = dt * L[0][1], a10 = dt * L[1][0], a11 = dt * L[1][1];
        detM = T(1) + ((a00 + a11) + (a00 * a11 - a01 * a10));
    }
    T dD = detM - T(1);
    T dJn = dJ + dD + dJ * dD;
    // s = -V0 J' p(J'),  p = (K/gamma)(J'^-gamma - 1)
    T Jmg = exp(-P.gamma * log1p(dJn));
    T dsdJ = -P.vol0 * P.k_over_gamma * ((T(1) - P.gamma) * Jmg - T(1));
    T Jb = Jb_out + sb_out * dsdJ;
    Jb_in = Jb * detM;
    T J = T(1) + dJ;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) Lb[i][j] = Jb * J * cof[i][j] * dt;
}

// Reverse of vfluid_update (Newtonian viscous fluid, Sec. 2.3
// eq:stress_strain): S = s_iso(J') I + c(J') (sym(L) - tr(L)/D I) with
// c = 2 mu V0 J' and s_iso the Tait part of fluid_update.  Inputs the
// step's velocity gradient L, the stored J - 1 and the adjoints Jb_out of
// J' - 1 and sb_out of the packed stress (an off-diagonal entry's adjoint is
// that of the packed value); outputs Lb and the adjoint Jb_in of J - 1.
template <class T, int D>
__device__ __forceinline__ void vfluid_vjp(const Phys<T>& P, const T L[D][D], T dJ, T Jb_out,
                                           const T sb_out[D * (D + 1) / 2], T Lb[D][D], T& Jb_in)
{
    T dJn = dJ, s_unused;
    fluid_update<T, D>(P, L, dJn, s_unused);
    const T c = T(2) * P.visc * P.vol0 * (T(1) + dJn);
    T trd = T(0), trs = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        trd += L[a][a];
        trs += sb_out[a];
    }
    // adjoint of c: <sb, sym(L) - tr(L)/D I> over the packed entries
    T cb = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int q = (i == j) ? i : (D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2);
            T r = T(0.5) * (L[i][j] + L[j][i]);
            if (i == j) r -= trd / T(D);
            cb += sb_out[q] * r;
        }
    fluid_vjp<T, D>(P, L, dJ, Jb_out + cb * T(2) * P.visc * P.vol0, trs, Lb, Jb_in);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (i == j) {
                Lb[i][i] += c * (sb_out[i] - trs / T(D));
            } else {
                const int q = D == 3 ? (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5)) : 2;
                Lb[i][j] += c * T(0.5) * sb_out[q];
            }
        }
}

// Reverse of wall_node for one face; vin is the velocity entering the face;
// vb is replaced by the adjoint of vin; returns dL/dmu.
template <class T, int D>
__device__ __forceinline__ T wall_node_vjp(int mode, T mu, int axis, T sign, const T vin[D], T vb[D])
{
    T vn = sign * vin[axis];
    if (!(vn > T(0))) return T(0);
    if (mode == WALL_STICK) {
#pragma unroll
        for (int a = 0; a < D; ++a) vb[a] = T(0);
        return T(0);
    }
    if (mode == WALL_SLIP) {
        vb[axis] = T(0);
        return T(0);
    }
    T vt[D], t2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        vt[a] = (a == axis) ? T(0) : vin[a];
        t2 += vt[a] * vt[a];
    }
    T t = sqrt(t2);
    if (t <= mu * vn) {
#pragma unroll
        for (int a = 0; a < D; ++a) vb[a] = T(0);
        return T(0);
    }
    T s = T(1) - mu * vn / t;
    T as = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) as += vb[a] * vt[a];
    T vtb[D];
#pragma unroll
    for (int a = 0; a < D; ++a) vtb[a] = s * vb[a] + as * mu * vn / (t * t * t) * vt[a];
    T vnb = -as * mu / t;
#pragma unroll
    for (int a = 0; a < D; ++a) vb[a] = (a == axis) ? sign * vnb : vtb[a];
    return -as * vn / t;
}

}  // namespace mpm
