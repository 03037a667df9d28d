/*
 * Reference adjoint of one MPM step, binary64 (TEST INFRASTRUCTURE ONLY).
 *
 * The paper differentiates the step map S^{t+1} = Phi(S^t; alpha) by reverse
 * mode (Sec. 3.1, eq:dzda; Sec. 3.2 the loss gradient).  This file writes
 * the vector-Jacobian product of one step of mpm_oracle.c by hand, stage by
 * stage in reverse: constitutive update, G2P, walls and grid update, P2G,
 * then the sort's permutation.  The constitutive part is built from its
 * Jacobian, column by column, with directional derivatives of the spectral
 * functions (the derivative of an isotropic matrix function in the
 * eigenbasis: divided differences f[l_i, l_j] off the diagonal, f'(l_i) on
 * it), so it shares no structure with a reverse-mode implementation.
 *
 * The sort permutation and wall/return-mapping case choices are held fixed
 * (they are piecewise constant); the clamp of positions into the domain
 * passes no gradient in a clamped component.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mpm_oracle.h"

/* second derivative of phi-bar (piecewise constant) */
static double ddphibar(double xi)
{
    double a = fabs(xi);
    if (a < 0.5) return -2.0;
    if (a < 1.5) return 1.0;
    return 0.0;
}

typedef struct {
    int32_t base[3];
    double w[3][3], dw[3][3], ddw[3][3];
} stencil2;

static void make_stencil2(const orc_config* c, const double* xp, stencil2* st)
{
    for (int a = 0; a < 3; ++a) {
        st->base[a] = 0;
        for (int k = 0; k < 3; ++k) {
            st->w[a][k] = (k == 0) ? 1.0 : 0.0;
            st->dw[a][k] = 0.0;
            st->ddw[a][k] = 0.0;
        }
    }
    for (int a = 0; a < c->dim; ++a) {
        orc_stencil_1d(xp[a], c->dx, c->key_f32, &st->base[a], st->w[a], st->dw[a]);
        double t = c->key_f32 ? (double)((float)xp[a] * (1.0f / (float)c->dx)) : xp[a] * (1.0 / c->dx);
        for (int k = 0; k < 3; ++k)
            st->ddw[a][k] = ddphibar(t - (double)(st->base[a] + k)) / (c->dx * c->dx);
    }
}

/* phi, grad phi, its Jacobian d(grad phi)/dx, dpos = x_i - x_p, node index */
static void node_terms(const orc_config* c, const double* xp, const stencil2* st, const int k[3],
                       double* phi, double g[3], double H[3][3], double dpos[3], int32_t I[3])
{
    int d = c->dim;
    double ph = 1.0;
    for (int a = 0; a < d; ++a) ph *= st->w[a][k[a]];
    *phi = ph;
    for (int a = 0; a < 3; ++a) {
        g[a] = 0.0;
        dpos[a] = 0.0;
        I[a] = 0;
        for (int b = 0; b < 3; ++b) H[a][b] = 0.0;
    }
    for (int a = 0; a < d; ++a) {
        double ga = st->dw[a][k[a]];
        for (int b = 0; b < d; ++b)
            if (b != a) ga *= st->w[b][k[b]];
        g[a] = ga;
        for (int cc = 0; cc < d; ++cc) {
            double h = 1.0;
            for (int b = 0; b < d; ++b) {
                if (b == a && b == cc) h *= st->ddw[b][k[b]];
                else if (b == a || b == cc) h *= st->dw[b][k[b]];
                else h *= st->w[b][k[b]];
            }
            H[a][cc] = h;
        }
        int32_t node = st->base[a] + k[a];
        dpos[a] = (double)node * c->dx - xp[a];
        I[a] = node + c->ghost;
    }
}

static int64_t lin3(const int32_t dims[3], const int32_t I[3])
{
    return ((int64_t)I[2] * dims[1] + I[1]) * dims[0] + I[0];
}

/* ------------------------------------------------------------------ */
/* Walls: forward with recorded inputs, and the vector-Jacobian product  */
/* ------------------------------------------------------------------ */

static void wall_fwd(int d, int mode, double mu, const double nrm[3], double vel[3])
{
    double vn = 0.0;
    for (int a = 0; a < d; ++a) vn += vel[a] * nrm[a];
    if (!(vn > 0.0)) return;
    double vt[3] = {0, 0, 0}, t2 = 0.0;
    for (int a = 0; a < d; ++a) {
        vt[a] = vel[a] - vn * nrm[a];
        t2 += vt[a] * vt[a];
    }
    if (mode == ORC_WALL_SLIP) {
        for (int a = 0; a < d; ++a) vel[a] = vt[a];
    } else if (mode == ORC_WALL_STICK) {
        for (int a = 0; a < d; ++a) vel[a] = 0.0;
    } else {
        double t = sqrt(t2);
        if (t <= mu * vn) {
            for (int a = 0; a < d; ++a) vel[a] = 0.0;
        } else {
            double s = 1.0 - mu * vn / t;
            for (int a = 0; a < d; ++a) vel[a] = vt[a] * s;
        }
    }
}

/* vin: velocity entering this face; vbar: adjoint of the face's output,
 * overwritten by the adjoint of its input; *mubar += dL/dmu. */
static void wall_vjp(int d, int mode, double mu, const double nrm[3], const double vin[3], double vbar[3],
                     double* mubar)
{
    double vn = 0.0;
    for (int a = 0; a < d; ++a) vn += vin[a] * nrm[a];
    if (!(vn > 0.0)) return;
    double vt[3] = {0, 0, 0}, t2 = 0.0;
    for (int a = 0; a < d; ++a) {
        vt[a] = vin[a] - vn * nrm[a];
        t2 += vt[a] * vt[a];
    }
    if (mode == ORC_WALL_STICK) {
        for (int a = 0; a < d; ++a) vbar[a] = 0.0;
        return;
    }
    if (mode == ORC_WALL_SLIP) {
        double p = 0.0;
        for (int a = 0; a < d; ++a) p += vbar[a] * nrm[a];
        for (int a = 0; a < d; ++a) vbar[a] -= p * nrm[a];
        return;
    }
    double t = sqrt(t2);
    if (t <= mu * vn) {
        for (int a = 0; a < d; ++a) vbar[a] = 0.0;
        return;
    }
    double s = 1.0 - mu * vn / t;
    double as = 0.0;
    for (int a = 0; a < d; ++a) as += vbar[a] * vt[a];
    double vtb[3];
    for (int a = 0; a < d; ++a) vtb[a] = s * vbar[a] + as * mu * vn / (t * t) * vt[a] / t;
    double vnb = -as * mu / t;
    if (mubar) *mubar += -as * vn / t;
    double p = 0.0;
    for (int a = 0; a < d; ++a) p += vtb[a] * nrm[a];
    for (int a = 0; a < d; ++a) vbar[a] = vtb[a] - p * nrm[a] + vnb * nrm[a];
}

/* ------------------------------------------------------------------ */
/* Spectral derivatives                                                 */
/* ------------------------------------------------------------------ */

/* divided difference of (1/2) ln at lambda_i, lambda_j */
static double dd_halflog(double li, double lj)
{
    double del = (li - lj) / lj;
    if (fabs(del) < 1e-4)
        return 0.5 / lj * (1.0 - del / 2.0 + del * del / 3.0 - del * del * del / 4.0);
    return 0.5 * log(li / lj) / (li - lj);
}

/* divided difference of exp at y_i, y_j */
static double dd_exp(double yi, double yj)
{
    double del = yi - yj;
    if (fabs(del) < 1e-5)
        return exp(yj) * (1.0 + del / 2.0 + del * del / 6.0);
    return exp(yj) * expm1(del) / del;
}

/* Y = U (K o (U^T A U)) U^T for the symmetric kernel K */
static void spectral_apply(int d, const double U[9], const double K[3][3], const double A[3][3], double Y[3][3])
{
    double B[3][3] = {{0}}, T[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int p = 0; p < d; ++p)
                for (int q = 0; q < d; ++q)
                    s += U[p * d + i] * A[p][q] * U[q * d + j];
            B[i][j] = s * K[i][j];
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int p = 0; p < d; ++p)
                for (int q = 0; q < d; ++q)
                    s += U[i * d + p] * B[p][q] * U[j * d + q];
            T[i][j] = s;
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Y[i][j] = T[i][j];
}

/* Directional derivative of the Hencky return (F_tr -> F_e', tau) at Ftr
 * along dF.  The case is the one the forward map takes at Ftr. */
static void hencky_tangent(const orc_config* c, int elastic_only, const double Ftr[3][3], const double dF[3][3],
                           double dFe[3][3], double dtau[3][3])
{
    int d = c->dim;
    double E = c->youngs, nu = c->poisson;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    double bm[9] = {0}, db[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0, t = 0.0;
            for (int k = 0; k < d; ++k) {
                s += Ftr[i][k] * Ftr[j][k];
                t += dF[i][k] * Ftr[j][k] + Ftr[i][k] * dF[j][k];
            }
            bm[i * d + j] = s;
            db[i][j] = t;
        }
    double lamv[3], U[9];
    orc_sym_eig(d, bm, lamv, U);
    double eps[3] = {0, 0, 0}, tr = 0.0;
    for (int i = 0; i < d; ++i) {
        eps[i] = 0.5 * log(lamv[i]);
        tr += eps[i];
    }
    double K[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            K[i][j] = (i == j) ? 0.5 / lamv[i] : dd_halflog(lamv[i], lamv[j]);
    double dE[3][3];
    spectral_apply(d, U, K, db, dE);
    double dtr = 0.0;
    for (int i = 0; i < d; ++i) dtr += dE[i][i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) { dFe[i][j] = 0.0; dtau[i][j] = 0.0; }

    /* case selection exactly as the forward map */
    double dev[3] = {0, 0, 0}, dn = 0.0;
    for (int i = 0; i < d; ++i) {
        dev[i] = eps[i] - tr / d;
        dn += dev[i] * dev[i];
    }
    dn = sqrt(dn);
    int cas;
    double alpha = orc_cone_alpha(c), cc = (d * lam + 2.0 * mu) / (2.0 * mu) * alpha;
    double en2 = 0.0;
    for (int i = 0; i < d; ++i) en2 += eps[i] * eps[i];
    if (elastic_only || en2 <= ORC_EPS_ELASTIC * ORC_EPS_ELASTIC) cas = 1;
    else if (tr > 0.0) cas = 0;
    else cas = (dn + cc * tr <= 0.0) ? 1 : 2;

    if (cas == 1) {
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                dFe[i][j] = dF[i][j];
                dtau[i][j] = 2.0 * mu * dE[i][j] + (i == j ? lam * dtr : 0.0);
            }
        return;
    }
    /* eigenvalues of Y (X = exp Y) and its tangent */
    double y[3] = {0, 0, 0}, dY[3][3] = {{0}};
    if (cas == 0) {
        for (int i = 0; i < d; ++i) y[i] = -eps[i];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) dY[i][j] = -dE[i][j];
    } else {
        /* Ehat = E - tr/d I; n = |Ehat|; kappa = 1 + cc tr / n; Y = -kappa Ehat */
        double kappa = 1.0 + cc * tr / dn;
        double Eh[3][3] = {{0}}, dEh[3][3] = {{0}};
        /* Ehat in the lab frame */
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double s = 0.0;
                for (int k = 0; k < d; ++k) s += U[i * d + k] * dev[k] * U[j * d + k];
                Eh[i][j] = s;
                dEh[i][j] = dE[i][j] - (i == j ? dtr / d : 0.0);
            }
        double dnn = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) dnn += Eh[i][j] * dEh[i][j];
        dnn /= dn;
        double dkappa = cc * (dtr * dn - tr * dnn) / (dn * dn);
        for (int i = 0; i < d; ++i) y[i] = -kappa * dev[i];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) dY[i][j] = -dkappa * Eh[i][j] - kappa * dEh[i][j];
        double a1 = 2.0 * mu / d + lam, b1 = 2.0 * mu * cc;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                dtau[i][j] = (i == j ? a1 * dtr : 0.0)
                           - b1 * (dtr * Eh[i][j] / dn + tr * dEh[i][j] / dn - tr * Eh[i][j] * dnn / (dn * dn));
    }
    double KX[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            KX[i][j] = (i == j) ? exp(y[i]) : dd_exp(y[i], y[j]);
    double dX[3][3];
    spectral_apply(d, U, KX, dY, dX);
    double X[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += U[i * d + k] * exp(y[k]) * U[j * d + k];
            X[i][j] = s;
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += dX[i][k] * Ftr[k][j] + X[i][k] * dF[k][j];
            dFe[i][j] = s;
        }
}

/* Directional derivative of the hypoelastic Drucker-Prager update of one
 * particle (Sec. 2.3 eq:dp_stress; App. A; the forward map is
 * orc_constitutive's DP_JAUMANN branch): inputs the stress cache S (V0 J
 * sigma), J and the velocity gradient L, outputs S' and J', along (dS, dJ,
 * dL).  The zone (and the corner of a shear return) is the one the forward
 * map takes at the point, read from orc_dp_jaumann itself. */
static void jaumann_tangent(const orc_config* c, double dt, const double S[3][3], double J, const double L[3][3],
                            const double dS[3][3], double dJ, const double dL[3][3], double dSo[3][3],
                            double* dJo)
{
    int d = c->dim;
    double E = c->youngs, nu = c->poisson;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double G = E / (2.0 * (1.0 + nu));
    double K = lam + 2.0 * G / d;
    double sp = sin(c->phi_deg * M_PI / 180.0), cp = cos(c->phi_deg * M_PI / 180.0);
    double ss = sin(c->psi_deg * M_PI / 180.0);
    double q_phi = 6.0 * sp / (sqrt(3.0) * (3.0 + sp));
    double k_phi = 6.0 * c->cohesion * cp / (sqrt(3.0) * (3.0 + sp));
    double q_psi = 6.0 * ss / (sqrt(3.0) * (3.0 + ss));
    double st = c->tension, tauP = k_phi - q_phi * st;

    /* volume: J' = J det(M), M = I + dt L; d det(M) = cof(M) : dM */
    double M[3][3] = {{0}}, cof[3][3] = {{0}};
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) M[a][b] = (a == b ? 1.0 : 0.0) + dt * L[a][b];
    double detM;
    if (d == 2) {
        detM = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        cof[0][0] = M[1][1]; cof[0][1] = -M[1][0];
        cof[1][0] = -M[0][1]; cof[1][1] = M[0][0];
    } else {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                cof[i][j] = M[i1][j1] * M[i2][j2] - M[i1][j2] * M[i2][j1];
            }
        detM = M[0][0] * cof[0][0] + M[0][1] * cof[0][1] + M[0][2] * cof[0][2];
    }
    double ddet = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) ddet += cof[a][b] * dt * dL[a][b];
    double Jn = J * detM, dJn = dJ * detM + J * ddet;

    /* Cauchy stress sigma = S / (V0 J) and its derivative */
    double sg[3][3] = {{0}}, dsg[3][3] = {{0}};
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            sg[a][b] = S[a][b] / (c->vol0 * J);
            dsg[a][b] = (dS[a][b] - sg[a][b] * c->vol0 * dJ) / (c->vol0 * J);
        }
    /* the zone the forward map takes */
    double Lf[9], sgf[9];
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            Lf[a * d + b] = L[a][b];
            sgf[a * d + b] = sg[a][b];
        }
    int zone = orc_dp_jaumann(c, dt, Lf, sgf, NULL);

    /* trial stress T and its derivative */
    double Dd[3][3] = {{0}}, Dw[3][3] = {{0}}, dDd[3][3] = {{0}}, dDw[3][3] = {{0}}, trD = 0.0, dtrD = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            Dd[a][b] = 0.5 * dt * (L[a][b] + L[b][a]);
            Dw[a][b] = 0.5 * dt * (L[a][b] - L[b][a]);
            dDd[a][b] = 0.5 * dt * (dL[a][b] + dL[b][a]);
            dDw[a][b] = 0.5 * dt * (dL[a][b] - dL[b][a]);
        }
    for (int a = 0; a < d; ++a) {
        trD += Dd[a][a];
        dtrD += dDd[a][a];
    }
    double T[3][3] = {{0}}, dT[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double r = sg[i][j], dr = dsg[i][j];
            for (int k = 0; k < d; ++k) {
                r += sg[i][k] * Dw[j][k] + sg[j][k] * Dw[i][k];
                dr += dsg[i][k] * Dw[j][k] + sg[i][k] * dDw[j][k] + dsg[j][k] * Dw[i][k] + sg[j][k] * dDw[i][k];
            }
            T[i][j] = r + 2.0 * G * Dd[i][j] + (i == j ? lam * trD : 0.0);
            dT[i][j] = dr + 2.0 * G * dDd[i][j] + (i == j ? lam * dtrD : 0.0);
        }
    double sm = 0.0, dsm = 0.0;
    for (int a = 0; a < d; ++a) {
        sm += T[a][a] / d;
        dsm += dT[a][a] / d;
    }
    double sv[3][3] = {{0}}, dsv[3][3] = {{0}}, ss2 = 0.0, sds = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            sv[i][j] = T[i][j] - (i == j ? sm : 0.0);
            dsv[i][j] = dT[i][j] - (i == j ? dsm : 0.0);
            ss2 += sv[i][j] * sv[i][j];
            sds += sv[i][j] * dsv[i][j];
        }
    double tau = sqrt(0.5 * ss2);
    double dtau = tau > 0.0 ? 0.5 * sds / tau : 0.0;      /* tau^2 = s:s/2 */

    double sm_n = sm, dsm_n = dsm, scale = 1.0, dscale = 0.0;
    if (zone == 2) {
        double fs = tau - k_phi + q_phi * sm, dfs = dtau + q_phi * dsm;
        double den = G + K * q_phi * q_psi;
        sm_n = sm - K * q_psi * fs / den;
        dsm_n = dsm - K * q_psi * dfs / den;
        double tau_n = k_phi - q_phi * sm_n, dtau_n = -q_phi * dsm_n;
        if (sm_n > st) {           /* the corner */
            sm_n = st;
            dsm_n = 0.0;
            tau_n = tauP;
            dtau_n = 0.0;
        }
        if (tau > 0.0) {
            scale = tau_n / tau;
            dscale = (dtau_n * tau - tau_n * dtau) / (tau * tau);
        } else {
            scale = 0.0;
            dscale = 0.0;
        }
    } else if (zone == 3) {
        sm_n = st;
        dsm_n = 0.0;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dSo[i][j] = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double so = scale * sv[i][j] + (i == j ? sm_n : 0.0);
            double dso = dscale * sv[i][j] + scale * dsv[i][j] + (i == j ? dsm_n : 0.0);
            dSo[i][j] = c->vol0 * (dJn * so + Jn * dso);
        }
    *dJo = dJn;
}

/* Directional derivative of the Newtonian fluid update of one particle
 * (Sec. 2.3 eq:stress_strain; the forward map is orc_constitutive's fluid
 * branch with orc_fluid_stress): inputs J and the velocity gradient L,
 * outputs J' = J det(I + dt L) and S' = V0 tau(J', L) with
 * tau = J' (-p(J') I + 2 mu (d - tr(d)/dim I)), d = (L + L^T)/2, along
 * (dJ, dL).  d det(M)[dM] = cof(M) : dM, and p'(J) = -K J^(-gamma-1). */
static void viscous_tangent(const orc_config* c, double dt, double J, const double L[3][3], double dJ,
                            const double dL[3][3], double dS[3][3], double* dJo)
{
    int d = c->dim;
    double M[3][3] = {{0}}, cof[3][3] = {{0}};
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) M[a][b] = (a == b ? 1.0 : 0.0) + dt * L[a][b];
    double detM;
    if (d == 2) {
        cof[0][0] = M[1][1]; cof[0][1] = -M[1][0];
        cof[1][0] = -M[0][1]; cof[1][1] = M[0][0];
        detM = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    } else {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                cof[i][j] = M[i1][j1] * M[i2][j2] - M[i1][j2] * M[i2][j1];
            }
        detM = M[0][0] * cof[0][0] + M[0][1] * cof[0][1] + M[0][2] * cof[0][2];
    }
    double ddet = 0.0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) ddet += cof[a][b] * dt * dL[a][b];
    double Jn = J * detM, dJn = dJ * detM + J * ddet;
    *dJo = dJn;
    double pr = orc_fluid_pressure(c, Jn);
    double dpr = -c->bulk * pow(Jn, -c->gamma - 1.0) * dJn;
    double tr = 0.0, dtr = 0.0;
    for (int a = 0; a < d; ++a) {
        tr += L[a][a];
        dtr += dL[a][a];
    }
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            double sig = 2.0 * c->viscosity * 0.5 * (L[a][b] + L[b][a]);
            double dsig = 2.0 * c->viscosity * 0.5 * (dL[a][b] + dL[b][a]);
            if (a == b) {
                sig += -pr - 2.0 * c->viscosity * tr / d;
                dsig += -dpr - 2.0 * c->viscosity * dtr / d;
            }
            dS[a][b] = c->vol0 * (dJn * sig + Jn * dsig);
        }
}

/* Which velocity component the resting obstacle o removes at node I moving
 * with vel (orc_obstacles' rule for one obstacle), or -1. */
static int obstacle_component(const orc_config* c, int o, const int32_t I[3], const double vel[3])
{
    int d = c->dim;
    double xi[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
        xi[a] = (double)(I[a] - c->ghost) * c->dx;
        if (xi[a] < c->obst_lo[o][a] || xi[a] > c->obst_hi[o][a]) return -1;
    }
    int best_a = -1, best_side = 0;
    double best = 0.0;
    for (int a = 0; a < d; ++a)
        for (int side = 0; side < 2; ++side) {
            double face = side == 0 ? c->obst_lo[o][a] : c->obst_hi[o][a];
            double ext = (double)c->n[a] * c->dx;
            if ((side == 0 && face <= 0.0) || (side == 1 && face >= ext)) continue;
            double depth = side == 0 ? xi[a] - face : face - xi[a];
            if (best_a < 0 || depth < best) {
                best = depth;
                best_a = a;
                best_side = side;
            }
        }
    if (best_a < 0) return -1;
    double vn = best_side == 0 ? vel[best_a] : -vel[best_a];
    return vn > 0.0 ? best_a : -1;
}

/* ------------------------------------------------------------------ */
/* One step's vector-Jacobian product                                   */
/* ------------------------------------------------------------------ */

int orc_adjoint_step(const orc_config* c, int64_t N, double dt, const double* floor_mu,
                     const double* x0, const double* v0, const double* C0, const double* F0,
                     const double* J0, const double* S0,
                     const double* ax1, const double* av1, const double* aC1, const double* aF1,
                     const double* aJ1, const double* aS1,
                     double* ax0, double* av0, double* aC0, double* aF0, double* aJ0, double* aS0,
                     double* amu)
{
    const int d = c->dim, dd = d * d;
    const int fluid = c->material == ORC_FLUID;
    const int jaumann = c->material == ORC_DP_JAUMANN;
    const int carries_j = fluid || jaumann;
    /* every transfer, resting obstacles, the (viscous) fluid, the Hencky
     * materials and the hypoelastic Drucker-Prager material */
    const int viscous = fluid && c->viscosity != 0.0;
    /* FLIP: v' = sum phi v_i + alpha (v_p - sum phi v_i^n) with the grid
     * velocity before the update v_i^n = Q_i / m_i, Q the momentum without
     * the internal force */
    const int flip = c->transfer == ORC_FLIP;
    int32_t dims[3];
    int64_t NN = orc_node_dims(c, dims);
    size_t NP = (size_t)(N > 0 ? N : 1);
    int32_t* key = malloc(sizeof(int32_t) * NP);
    int32_t* perm = malloc(sizeof(int32_t) * NP);
    double* X = malloc(sizeof(double) * NP * d);
    double* V = malloc(sizeof(double) * NP * d);
    double* Cm = malloc(sizeof(double) * NP * dd);
    double* Fm = malloc(sizeof(double) * NP * dd);
    double* Jm = malloc(sizeof(double) * NP);
    double* Sm = malloc(sizeof(double) * NP * dd);
    double* gm = calloc((size_t)NN, sizeof(double));
    double* gp = calloc((size_t)NN * d, sizeof(double));
    double* gvt = calloc((size_t)NN * d, sizeof(double));  /* before walls */
    double* gv = calloc((size_t)NN * d, sizeof(double));   /* after walls */
    double* gvb = calloc((size_t)NN * d, sizeof(double));  /* adjoint of gv */
    double* gmb = calloc((size_t)NN, sizeof(double));      /* adjoint of m */
    double* gpb = calloc((size_t)NN * d, sizeof(double));  /* adjoint of P */
    double* gq = calloc((size_t)NN * d, sizeof(double));   /* FLIP: Q, then v^n = Q / m */
    double* gvob = calloc((size_t)NN * d, sizeof(double)); /* FLIP: adjoint of v^n */
    double* gqb = calloc((size_t)NN * d, sizeof(double));  /* FLIP: adjoint of Q */
    double* axs = calloc(NP * d, sizeof(double));          /* sorted-order adjoints */
    double* avs = calloc(NP * d, sizeof(double));
    double* aCs = calloc(NP * dd, sizeof(double));
    double* aFs = calloc(NP * dd, sizeof(double));
    double* aJs = calloc(NP, sizeof(double));
    double* aSs = calloc(NP * dd, sizeof(double));
    if (!key || !perm || !X || !V || !Cm || !Fm || !Jm || !Sm || !gm || !gp || !gvt || !gv || !gvb || !gmb ||
        !gpb || !gq || !gvob || !gqb || !axs || !avs || !aCs || !aFs || !aJs || !aSs)
        return -1;

    /* the step's sort, applied to a copy of the input state */
    orc_cell_keys(c, N, x0, key);
    orc_sort_perm(N, key, orc_cells_per_tile(c), perm);
    for (int64_t s = 0; s < N; ++s) {
        int64_t j = perm[s];
        for (int a = 0; a < d; ++a) {
            X[a * N + s] = x0[a * N + j];
            V[a * N + s] = v0[a * N + j];
        }
        for (int q = 0; q < dd; ++q) {
            Cm[q * N + s] = C0[q * N + j];
            Fm[q * N + s] = carries_j ? 0.0 : F0[q * N + j];
            Sm[q * N + s] = S0[q * N + j];
        }
        Jm[s] = carries_j ? J0[j] : 1.0;
    }

    /* forward recomputation: P2G and grid (velocity before and after walls) */
    orc_p2g_ex(c, N, dt, X, V, Cm, Sm, gm, gp, flip ? gq : NULL);
    if (flip)
        for (int64_t i = 0; i < NN; ++i)
            for (int a = 0; a < d; ++a) gq[a * NN + i] = gm[i] > 0.0 ? gq[a * NN + i] / gm[i] : 0.0;
    int fl = d - 1;
    for (int32_t Iz = 0; Iz < dims[2]; ++Iz)
        for (int32_t Iy = 0; Iy < dims[1]; ++Iy)
            for (int32_t Ix = 0; Ix < dims[0]; ++Ix) {
                int32_t I[3] = {Ix, Iy, Iz};
                int64_t li = lin3(dims, I);
                double vel[3] = {0, 0, 0};
                if (gm[li] > 0.0)
                    for (int a = 0; a < d; ++a) vel[a] = gp[a * NN + li] / gm[li] + dt * c->gravity[a];
                for (int a = 0; a < d; ++a) gvt[a * NN + li] = vel[a];
                if (gm[li] > 0.0) {
                    for (int a = 0; a < d; ++a) {
                        int32_t i = I[a] - c->ghost;
                        for (int side = 0; side < 2; ++side) {
                            int beyond = side == 0 ? (i <= 0) : (i >= c->n[a]);
                            if (!beyond) continue;
                            double nrm[3] = {0, 0, 0};
                            nrm[a] = side == 0 ? -1.0 : 1.0;
                            double mu = c->wall_mu[2 * a + side];
                            if (floor_mu && a == fl && side == 0)
                                mu = floor_mu[(d == 3) ? ((int64_t)Iy * dims[0] + Ix) : Ix];
                            wall_fwd(d, c->wall_mode[2 * a + side], mu, nrm, vel);
                        }
                    }
                    for (int o = 0; o < c->n_obstacles; ++o) {
                        int a = obstacle_component(c, o, I, vel);
                        if (a >= 0) vel[a] = 0.0;
                    }
                }
                for (int a = 0; a < d; ++a) gv[a * NN + li] = vel[a];
            }

    double Dinv = 4.0 / (c->dx * c->dx);
    int kz_max = (d == 3) ? 3 : 1;

    /* --- reverse of the constitutive update and of G2P, per particle --- */
    for (int64_t s = 0; s < N; ++s) {
        double xp[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) xp[a] = X[a * N + s];
        stencil2 st;
        make_stencil2(c, xp, &st);
        /* forward G2P */
        double vn[3] = {0, 0, 0}, Bm[3][3] = {{0}}, L[3][3] = {{0}};
        for (int k2 = 0; k2 < kz_max; ++k2)
            for (int k1 = 0; k1 < 3; ++k1)
                for (int k0 = 0; k0 < 3; ++k0) {
                    int k[3] = {k0, k1, k2};
                    double phi, g[3], H[3][3], dp[3];
                    int32_t I[3];
                    node_terms(c, xp, &st, k, &phi, g, H, dp, I);
                    int64_t li = lin3(dims, I);
                    for (int a = 0; a < d; ++a) {
                        double vi = gv[a * NN + li];
                        vn[a] += phi * vi;
                        for (int b = 0; b < d; ++b) {
                            Bm[a][b] += phi * vi * dp[b];
                            L[a][b] += vi * g[b];
                        }
                    }
                }
        double M[3][3] = {{0}};
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) M[a][b] = (a == b ? 1.0 : 0.0) + dt * L[a][b];

        /* adjoint of the constitutive outputs -> Lbar and the input F/J adjoint */
        double Lb[3][3] = {{0}};
        if (jaumann) {
            /* contract the output adjoints (S', J') with the tangent along
             * every input direction: S entries, J, L entries */
            double Sp[3][3] = {{0}}, Lp[3][3] = {{0}}, zero[3][3] = {{0}}, dSo[3][3];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    Sp[a][b] = Sm[(a * d + b) * N + s];
                    Lp[a][b] = L[a][b];
                }
            double dJo;
            for (int p = 0; p < d; ++p)
                for (int q = 0; q < d; ++q) {
                    double e[3][3] = {{0}};
                    e[p][q] = 1.0;
                    double sum;
                    /* along S_pq: the constitutive part of the input stress adjoint */
                    jaumann_tangent(c, dt, Sp, Jm[s], Lp, e, 0.0, zero, dSo, &dJo);
                    sum = aJ1[s] * dJo;
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b) sum += aS1[(a * d + b) * N + s] * dSo[a][b];
                    aSs[(p * d + q) * N + s] += sum;
                    /* along L_pq */
                    jaumann_tangent(c, dt, Sp, Jm[s], Lp, zero, 0.0, e, dSo, &dJo);
                    sum = aJ1[s] * dJo;
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b) sum += aS1[(a * d + b) * N + s] * dSo[a][b];
                    Lb[p][q] = sum;
                }
            jaumann_tangent(c, dt, Sp, Jm[s], Lp, zero, 1.0, zero, dSo, &dJo);
            double sum = aJ1[s] * dJo;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) sum += aS1[(a * d + b) * N + s] * dSo[a][b];
            aJs[s] = sum;
        } else if (viscous) {
            /* contract the output adjoints (S', J') with the tangent along
             * every input direction: J and the L entries */
            double Lp[3][3] = {{0}}, zero[3][3] = {{0}}, dSo[3][3], dJo;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) Lp[a][b] = L[a][b];
            for (int p = 0; p < d; ++p)
                for (int q = 0; q < d; ++q) {
                    double e[3][3] = {{0}};
                    e[p][q] = 1.0;
                    viscous_tangent(c, dt, Jm[s], Lp, 0.0, e, dSo, &dJo);
                    double sum = aJ1[s] * dJo;
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b) sum += aS1[(a * d + b) * N + s] * dSo[a][b];
                    Lb[p][q] = sum;
                }
            viscous_tangent(c, dt, Jm[s], Lp, 1.0, zero, dSo, &dJo);
            double sum = aJ1[s] * dJo;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) sum += aS1[(a * d + b) * N + s] * dSo[a][b];
            aJs[s] = sum;
        } else if (fluid) {
            double detM = (d == 2) ? M[0][0] * M[1][1] - M[0][1] * M[1][0]
                                   : M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                                   - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                                   + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            double Jn = Jm[s] * detM;
            /* S' = -V0 J' p(J') I, p = (K/g)(J'^-g - 1) */
            double trSb = 0.0;
            for (int a = 0; a < d; ++a) trSb += aS1[(a * d + a) * N + s];
            double dsdJ = -c->vol0 * (c->bulk / c->gamma) * ((1.0 - c->gamma) * pow(Jn, -c->gamma) - 1.0);
            double Jb = aJ1[s] + trSb * dsdJ;
            aJs[s] = Jb * detM;
            /* d det(M) / dM = cofactor(M) */
            double cof[3][3] = {{0}};
            if (d == 2) {
                cof[0][0] = M[1][1]; cof[0][1] = -M[1][0];
                cof[1][0] = -M[0][1]; cof[1][1] = M[0][0];
            } else {
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                        cof[i][j] = M[i1][j1] * M[i2][j2] - M[i1][j2] * M[i2][j1];
                    }
            }
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) Lb[a][b] = Jb * Jm[s] * cof[a][b] * dt;
        } else {
            double Fo[3][3] = {{0}}, Ft[3][3] = {{0}};
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) Fo[a][b] = Fm[(a * d + b) * N + s];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double t = 0.0;
                    for (int k = 0; k < d; ++k) t += M[a][k] * Fo[k][b];
                    Ft[a][b] = t;
                }
            /* Ftr bar: contract output adjoints with each Jacobian column */
            double Ftb[3][3] = {{0}};
            for (int p = 0; p < d; ++p)
                for (int q = 0; q < d; ++q) {
                    double dF[3][3] = {{0}}, dFe[3][3], dtau[3][3];
                    dF[p][q] = 1.0;
                    hencky_tangent(c, c->material == ORC_HENCKY_ELASTIC, Ft, dF, dFe, dtau);
                    double sum = 0.0;
                    for (int a = 0; a < d; ++a)
                        for (int b = 0; b < d; ++b)
                            sum += aF1[(a * d + b) * N + s] * dFe[a][b]
                                 + aS1[(a * d + b) * N + s] * c->vol0 * dtau[a][b];
                    Ftb[p][q] = sum;
                }
            /* Ftr = M Fo: Lbar = dt Ftb Fo^T, Fo bar = M^T Ftb */
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    double l = 0.0, f = 0.0;
                    for (int k = 0; k < d; ++k) {
                        l += Ftb[a][k] * Fo[b][k];
                        f += M[k][a] * Ftb[k][b];
                    }
                    Lb[a][b] = dt * l;
                    aFs[(a * d + b) * N + s] = f;
                }
        }

        /* FLIP: the particle's own velocity and the gathered v^n */
        double vob[3] = {0, 0, 0};
        if (flip)
            for (int a = 0; a < d; ++a) {
                avs[a * N + s] += c->flip_alpha * av1[a * N + s];
                vob[a] = -c->flip_alpha * av1[a * N + s];
            }
        /* positions: x' = clamp(x + dt sum phi v_i) */
        double vb[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            vb[a] = av1[a * N + s];
            double xn = xp[a] + dt * vn[a];
            double hi = (double)c->n[a] * c->dx;
            if (xn >= 0.0 && xn <= hi) {
                axs[a * N + s] += ax1[a * N + s];
                vb[a] += dt * ax1[a * N + s];
            }
        }
        /* the carried matrix: APIC's C' = Dinv sum phi v_i (x_i - x_p)^T,
         * TPIC's C' = L (its adjoint joins the constitutive L adjoint),
         * PIC's C' = 0 (no adjoint flows back) */
        const int apic = c->transfer == ORC_APIC;
        if (c->transfer == ORC_TPIC)
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) Lb[a][b] += aC1[(a * d + b) * N + s];
        /* G2P reverse */
        for (int k2 = 0; k2 < kz_max; ++k2)
            for (int k1 = 0; k1 < 3; ++k1)
                for (int k0 = 0; k0 < 3; ++k0) {
                    int k[3] = {k0, k1, k2};
                    double phi, g[3], H[3][3], dp[3];
                    int32_t I[3];
                    node_terms(c, xp, &st, k, &phi, g, H, dp, I);
                    int64_t li = lin3(dims, I);
                    double wb = 0.0, gb[3] = {0, 0, 0}, db[3] = {0, 0, 0};
                    for (int a = 0; a < d; ++a) {
                        double vi = gv[a * NN + li];
                        double acc = phi * vb[a];
                        wb += vi * vb[a];
                        if (flip) {
                            gvob[a * NN + li] += phi * vob[a];
                            wb += gq[a * NN + li] * vob[a];
                        }
                        for (int b = 0; b < d; ++b) {
                            double cb = apic ? aC1[(a * d + b) * N + s] : 0.0;
                            acc += Dinv * phi * cb * dp[b] + Lb[a][b] * g[b];
                            wb += Dinv * cb * vi * dp[b];
                            db[b] += Dinv * phi * cb * vi;
                            gb[b] += Lb[a][b] * vi;
                        }
                        gvb[a * NN + li] += acc;
                    }
                    for (int cc = 0; cc < d; ++cc) {
                        double t = wb * g[cc] - db[cc];
                        for (int b = 0; b < d; ++b) t += gb[b] * H[b][cc];
                        axs[cc * N + s] += t;
                    }
                }
    }

    /* --- reverse of the walls and the grid update --- */
    for (int32_t Iz = 0; Iz < dims[2]; ++Iz)
        for (int32_t Iy = 0; Iy < dims[1]; ++Iy)
            for (int32_t Ix = 0; Ix < dims[0]; ++Ix) {
                int32_t I[3] = {Ix, Iy, Iz};
                int64_t li = lin3(dims, I);
                double m = gm[li];
                if (!(m > 0.0)) continue;
                /* replay the faces, keeping each face's input velocity */
                double vin[6][3], vel[3] = {0, 0, 0};
                int face_of[6], nf = 0;
                double mu_of[6];
                for (int a = 0; a < d; ++a) vel[a] = gvt[a * NN + li];
                for (int a = 0; a < d; ++a) {
                    int32_t i = I[a] - c->ghost;
                    for (int side = 0; side < 2; ++side) {
                        int beyond = side == 0 ? (i <= 0) : (i >= c->n[a]);
                        if (!beyond) continue;
                        double nrm[3] = {0, 0, 0};
                        nrm[a] = side == 0 ? -1.0 : 1.0;
                        double mu = c->wall_mu[2 * a + side];
                        if (floor_mu && a == fl && side == 0)
                            mu = floor_mu[(d == 3) ? ((int64_t)Iy * dims[0] + Ix) : Ix];
                        for (int q = 0; q < 3; ++q) vin[nf][q] = vel[q];
                        face_of[nf] = 2 * a + side;
                        mu_of[nf] = mu;
                        ++nf;
                        wall_fwd(d, c->wall_mode[2 * a + side], mu, nrm, vel);
                    }
                }
                /* the obstacles, after the walls: each keeps its input velocity */
                double vob[ORC_MAX_OBSTACLES][3];
                for (int o = 0; o < c->n_obstacles; ++o) {
                    for (int q = 0; q < 3; ++q) vob[o][q] = vel[q];
                    int a = obstacle_component(c, o, I, vel);
                    if (a >= 0) vel[a] = 0.0;
                }
                double vbar[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a) vbar[a] = gvb[a * NN + li];
                /* a removed component passes no adjoint back */
                for (int o = c->n_obstacles - 1; o >= 0; --o) {
                    int a = obstacle_component(c, o, I, vob[o]);
                    if (a >= 0) vbar[a] = 0.0;
                }
                for (int f = nf - 1; f >= 0; --f) {
                    int face = face_of[f], a = face / 2;
                    double nrm[3] = {0, 0, 0};
                    nrm[a] = (face % 2 == 0) ? -1.0 : 1.0;
                    double mub = 0.0;
                    wall_vjp(d, c->wall_mode[face], mu_of[f], nrm, vin[f], vbar, &mub);
                    if (amu && floor_mu && a == fl && face % 2 == 0)
                        amu[(d == 3) ? ((int64_t)Iy * dims[0] + Ix) : Ix] += mub;
                }
                /* v~ = P/m + dt g; FLIP: v^n = Q/m */
                double dotv = 0.0;
                for (int a = 0; a < d; ++a) {
                    gpb[a * NN + li] = vbar[a] / m;
                    dotv += vbar[a] * (gvt[a * NN + li] - dt * c->gravity[a]);
                    if (flip) {
                        gqb[a * NN + li] = gvob[a * NN + li] / m;
                        dotv += gvob[a * NN + li] * gq[a * NN + li];
                    }
                }
                gmb[li] = -dotv / m;
            }

    /* --- reverse of P2G, per particle --- */
    for (int64_t s = 0; s < N; ++s) {
        double xp[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            xp[a] = X[a * N + s];
            vp[a] = V[a * N + s];
        }
        stencil2 st;
        make_stencil2(c, xp, &st);
        for (int k2 = 0; k2 < kz_max; ++k2)
            for (int k1 = 0; k1 < 3; ++k1)
                for (int k0 = 0; k0 < 3; ++k0) {
                    int k[3] = {k0, k1, k2};
                    double phi, g[3], H[3][3], dp[3];
                    int32_t I[3];
                    node_terms(c, xp, &st, k, &phi, g, H, dp, I);
                    int64_t li = lin3(dims, I);
                    double wb = c->mass * gmb[li];
                    double gb[3] = {0, 0, 0}, db[3] = {0, 0, 0};
                    for (int a = 0; a < d; ++a) {
                        double pb = gpb[a * NN + li];
                        /* FLIP's Q shares P's affine momentum, not its force */
                        double ab = flip ? pb + gqb[a * NN + li] : pb;
                        double aff = vp[a];
                        for (int b = 0; b < d; ++b) aff += Cm[(a * d + b) * N + s] * dp[b];
                        wb += c->mass * aff * ab;
                        avs[a * N + s] += phi * c->mass * ab;
                        for (int b = 0; b < d; ++b) {
                            aCs[(a * d + b) * N + s] += phi * c->mass * ab * dp[b];
                            db[b] += phi * c->mass * Cm[(a * d + b) * N + s] * ab;
                            aSs[(a * d + b) * N + s] += -dt * pb * g[b];
                            gb[b] += -dt * Sm[(a * d + b) * N + s] * pb;
                        }
                    }
                    for (int cc = 0; cc < d; ++cc) {
                        double t = wb * g[cc] - db[cc];
                        for (int b = 0; b < d; ++b) t += gb[b] * H[b][cc];
                        axs[cc * N + s] += t;
                    }
                }
    }

    /* --- undo the sort: adjoint of slot s goes to the particle's input slot --- */
    for (int64_t s = 0; s < N; ++s) {
        int64_t j = perm[s];
        for (int a = 0; a < d; ++a) {
            ax0[a * N + j] = axs[a * N + s];
            av0[a * N + j] = avs[a * N + s];
        }
        for (int q = 0; q < dd; ++q) {
            aC0[q * N + j] = aCs[q * N + s];
            aS0[q * N + j] = aSs[q * N + s];
            if (!carries_j) aF0[q * N + j] = aFs[q * N + s];
        }
        if (carries_j) aJ0[j] = aJs[s];
    }

    free(key); free(perm); free(X); free(V); free(Cm); free(Fm); free(Jm); free(Sm);
    free(gm); free(gp); free(gvt); free(gv); free(gvb); free(gmb); free(gpb); free(gq); free(gvob); free(gqb);
    free(axs); free(avs); free(aCs); free(aFs); free(aJs); free(aSs);
    return 0;
}
