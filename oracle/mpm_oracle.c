/*
 * Reference explicit MPM step in binary64, written for checking only.
 *
 * TEST INFRASTRUCTURE: this file is the oracle.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the HIP library: it is written from
 * the paper's equations, one stage per function, with plain scalar loops.
 *
 * Paper: "JAX-MPM: A Learning-Augmented Differentiable Meshfree Framework"
 * (Du & He, arXiv 2507.04192).
 *   - quadratic B-spline basis                 Sec. 2.1, eq. for phi-bar
 *   - lumped mass, explicit Euler              Sec. 2.1, eq:semi_eq
 *   - P2G / grid update / G2P (USL order)      Sec. 2.2
 *   - APIC transfer, D_p^{-1} = 4/h^2 I        App. B
 *   - weakly compressible EOS                  Sec. 2.3, eq:eos (Tait form)
 *   - Drucker-Prager cone slope q_phi          App. A
 *   - Coulomb wall friction                    Sec. 5.3, eq:coulomb_friction
 *   - Hencky-strain return on the D-P cone     (Klar et al. 2016, cited in
 *                                               Sec. 4.2.3)
 *   - FLIP, PIC, their blend, TPIC transfers   Sec. 2.2 G2P, App. B
 *   - Newtonian viscous stress                 Sec. 2.3, eq:stress_strain
 *   - hypoelastic Drucker-Prager with the
 *     Jaumann rate and tension cutoff          Sec. 2.3 eq:dp_stress, App. A
 *   - resting rigid obstacles, frictionless
 *     contact (normal velocity removed)        Sec. 4.2.1
 *
 * Readings taken where the paper is silent (all listed with reasons in the
 * design notes):
 *   - node i sits at i*h, i in [-G, n+G]; stored index I = i + G;
 *   - stencil base b = floor(fl(x*inv) - 0.5), inv = 1/h rounded once;
 *   - particles are clamped into [0, n*h] after advection;
 *   - walls: every node on or beyond a wall plane, faces in the order
 *     x-, x+, y-, y+, z-, z+; act only when the normal velocity points into
 *     the wall; slip / stick / Coulomb(mu);
 *   - fluid: p = (K/gamma)((1/J)^gamma - 1), J' = J det(I + dt L);
 *   - sand: Hencky strain of b = F F^T, radial return onto the cone
 *     ||dev eps|| + alpha (d lam + 2 mu)/(2 mu) tr eps <= 0 with
 *     alpha = (sqrt 2 / 3) q_phi, apex when tr eps > 0;
 *   - cell key: tile-major linear index of the stencil base, so that a
 *     stable sort by key groups particles by tile, then by cell.
 *
 * Arrays are structure-of-arrays, component-major: component a of particle p
 * is at arr[a*N + p]; a d x d matrix entry (a,b) is at arr[(a*d+b)*N + p].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mpm_oracle.h"

/* The number type of the particle and grid data, orc_real, is binary64
 * (double) in the oracle proper.  Built with ORC_COMPLEX_STEP it is a
 * complex binary64 number instead, for the complex-step derivative
 * f'(a) delta = Im f(a + i h delta) / h of the adjoint's checks: every
 * branch is then taken on the real part and the functions below are the
 * analytic continuations of the real ones. */
#ifdef ORC_COMPLEX_STEP
#define RE(a) creal(a)
#define ABS(a) (creal(a) < 0.0 ? -(a) : (a))
#define SQRT csqrt
#define LOG clog
#define EXP cexp
#define POW cpow
#else
#define RE(a) (a)
#define ABS fabs
#define SQRT sqrt
#define LOG log
#define EXP exp
#define POW pow
#endif

/* ------------------------------------------------------------------ */
/* Quadratic B-spline (Sec. 2.1, the piecewise definition of phi-bar) */
/* ------------------------------------------------------------------ */

orc_real orc_phibar(orc_real xi)
{
    orc_real a = ABS(xi);
    if (RE(a) < 0.5)
        return 0.75 - a * a;
    if (RE(a) < 1.5)
        return 0.5 * a * a - 1.5 * a + 1.125;
    return 0.0;
}

/* d phibar / d xi */
orc_real orc_dphibar(orc_real xi)
{
    orc_real a = ABS(xi);
    double s = (RE(xi) < 0.0) ? -1.0 : 1.0;
    if (RE(a) < 0.5)
        return -2.0 * xi;
    if (RE(a) < 1.5)
        return s * (a - 1.5);
    return 0.0;
}

/* Base node and the three 1-D weights / derivatives (per unit length) for
 * one coordinate.  key_f32 selects binary32 for t = x*inv so that keys can
 * be compared bit for bit with a binary32 solver. */
void orc_stencil_1d(orc_real x, double h, int key_f32, int32_t* base,
                    orc_real w[3], orc_real dw[3])
{
    orc_real t;
    if (key_f32) {
        float invf = 1.0f / (float)h;
        float tf = (float)RE(x) * invf;
        t = (orc_real)tf;
#ifdef ORC_COMPLEX_STEP
        t += cimag(x) * (1.0 / h) * _Complex_I;
#endif
    } else {
        double inv = 1.0 / h;
        t = x * inv;
    }
    int32_t b = (int32_t)floor(RE(t) - 0.5);
    *base = b;
    for (int k = 0; k < 3; ++k) {
        orc_real xi = t - (orc_real)(b + k); /* (x - x_i)/h */
        w[k] = orc_phibar(xi);
        dw[k] = orc_dphibar(xi) / h;
    }
}

/* ------------------------------------------------------------------ */
/* Grid bookkeeping                                                    */
/* ------------------------------------------------------------------ */

static int dimv(const orc_config* c) { return c->dim; }

int64_t orc_node_dims(const orc_config* c, int32_t dims[3])
{
    int64_t nn = 1;
    for (int a = 0; a < 3; ++a) {
        dims[a] = (a < c->dim) ? c->n[a] + 1 + 2 * c->ghost : 1;
        nn *= dims[a];
    }
    return nn;
}

static int64_t node_lin(const int32_t dims[3], const int32_t I[3])
{
    return ((int64_t)I[2] * dims[1] + I[1]) * dims[0] + I[0];
}

/* ------------------------------------------------------------------ */
/* Cell key and stable sort                                            */
/* ------------------------------------------------------------------ */

int64_t orc_num_keys(const orc_config* c)
{
    int64_t k = 1;
    for (int a = 0; a < c->dim; ++a) {
        int32_t span = c->n[a] + 2 * c->ghost + 1; /* possible B values */
        int32_t nt = (span + c->tile - 1) / c->tile;
        k *= (int64_t)nt * c->tile;
    }
    return k;
}

/* Key of a base index triple B (= base + ghost): tiles ordered x fastest,
 * then cells inside the tile ordered x fastest. */
int64_t orc_key_of_base(const orc_config* c, const int32_t B[3])
{
    int d = c->dim, T = c->tile;
    int64_t tile_lin = 0, cell_lin = 0, tiles_stride = 1, cells_stride = 1;
    for (int a = 0; a < d; ++a) {
        int32_t span = c->n[a] + 2 * c->ghost + 1;
        int32_t nt = (span + T - 1) / T;
        tile_lin += (int64_t)(B[a] / T) * tiles_stride;
        cell_lin += (int64_t)(B[a] % T) * cells_stride;
        tiles_stride *= nt;
        cells_stride *= T;
    }
    return tile_lin * cells_stride + cell_lin;
}

void orc_cell_keys(const orc_config* c, int64_t N, const orc_real* x, int32_t* key)
{
    int d = dimv(c);
    for (int64_t p = 0; p < N; ++p) {
        int32_t B[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            int32_t b;
            orc_real w[3], dw[3];
            orc_stencil_1d(x[a * N + p], c->dx, c->key_f32, &b, w, dw);
            B[a] = b + c->ghost;
        }
        key[p] = (int32_t)orc_key_of_base(c, B);
    }
}

typedef struct { int32_t key; int32_t slot; } keyslot;

static int cmp_keyslot(const void* pa, const void* pb)
{
    const keyslot* a = (const keyslot*)pa;
    const keyslot* b = (const keyslot*)pb;
    if (a->key != b->key) return (a->key < b->key) ? -1 : 1;
    if (a->slot != b->slot) return (a->slot < b->slot) ? -1 : 1;
    return 0;
}

/* Sort order of a step.  Particles are grouped by tile (key / cpt, with
 * cpt = cells per tile = T^d); inside a tile they are ordered by their rank
 * within their cell (the number of particles of the same key at smaller
 * current slots), then by the cell (key % cpt).  So the r-th particles of
 * all cells of a tile sit next to each other.  Computed in two plain
 * passes: a sort by (key, slot) gives the ranks, a sort by (tile, rank,
 * cell) the order. */
typedef struct {
    int32_t tile, rank, cell, slot;
} trc;

static int cmp_trc(const void* a, const void* b)
{
    const trc* x = (const trc*)a;
    const trc* y = (const trc*)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->rank != y->rank) return x->rank < y->rank ? -1 : 1;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return 0;
}

int32_t orc_cells_per_tile(const orc_config* c)
{
    int32_t k = 1;
    for (int a = 0; a < c->dim; ++a) k *= c->tile;
    return k;
}

void orc_sort_perm(int64_t N, const int32_t* key, int32_t cpt, int32_t* perm)
{
    size_t n1 = (size_t)(N > 0 ? N : 1);
    keyslot* ks = (keyslot*)malloc(sizeof(keyslot) * n1);
    trc* t = (trc*)malloc(sizeof(trc) * n1);
    for (int64_t p = 0; p < N; ++p) {
        ks[p].key = key[p];
        ks[p].slot = (int32_t)p;
    }
    qsort(ks, (size_t)N, sizeof(keyslot), cmp_keyslot);
    int32_t rank = 0;
    for (int64_t s = 0; s < N; ++s) {
        rank = (s > 0 && ks[s].key == ks[s - 1].key) ? rank + 1 : 0;
        t[s].tile = ks[s].key / cpt;
        t[s].cell = ks[s].key % cpt;
        t[s].rank = rank;
        t[s].slot = ks[s].slot;
    }
    qsort(t, (size_t)N, sizeof(trc), cmp_trc);
    for (int64_t s = 0; s < N; ++s)
        perm[s] = t[s].slot;
    free(t);
    free(ks);
}

static void gather_d(int64_t N, int ncomp, orc_real* a, const int32_t* perm, orc_real* tmp)
{
    for (int c = 0; c < ncomp; ++c) {
        for (int64_t s = 0; s < N; ++s)
            tmp[s] = a[c * N + perm[s]];
        memcpy(a + c * N, tmp, sizeof(orc_real) * (size_t)N);
    }
}

static void gather_i(int64_t N, int32_t* a, const int32_t* perm, int32_t* tmp)
{
    for (int64_t s = 0; s < N; ++s)
        tmp[s] = a[perm[s]];
    memcpy(a, tmp, sizeof(int32_t) * (size_t)N);
}

/* ------------------------------------------------------------------ */
/* P2G (Sec. 2.2 eq:update_m, momentum, force; App. B APIC)            */
/* ------------------------------------------------------------------ */

/* Per-particle stencil: node indices and phi, grad phi, x_i - x_p. */
typedef struct {
    int32_t base[3];
    orc_real w[3][3];  /* [axis][k] */
    orc_real dw[3][3];
} stencil;

static void make_stencil(const orc_config* c, int64_t N, const orc_real* x, int64_t p, stencil* st)
{
    for (int a = 0; a < 3; ++a) {
        st->base[a] = 0;
        for (int k = 0; k < 3; ++k) {
            st->w[a][k] = (k == 0) ? 1.0 : 0.0;
            st->dw[a][k] = 0.0;
        }
    }
    for (int a = 0; a < c->dim; ++a) {
        orc_stencil_1d(x[a * N + p], c->dx, c->key_f32, &st->base[a], st->w[a], st->dw[a]);
    }
}

/* For stencil offset (k0,k1,k2): phi, grad phi and dpos = x_i - x_p. */
static void stencil_node(const orc_config* c, const orc_real* xp, const stencil* st,
                         const int k[3], orc_real* phi, orc_real grad[3], orc_real dpos[3], int32_t I[3])
{
    int d = c->dim;
    orc_real ph = 1.0;
    for (int a = 0; a < d; ++a)
        ph *= st->w[a][k[a]];
    *phi = ph;
    for (int a = 0; a < 3; ++a) {
        grad[a] = 0.0;
        dpos[a] = 0.0;
        I[a] = 0;
    }
    for (int a = 0; a < d; ++a) {
        orc_real g = st->dw[a][k[a]];
        for (int b = 0; b < d; ++b)
            if (b != a) g *= st->w[b][k[b]];
        grad[a] = g;
        int32_t node = st->base[a] + k[a];
        dpos[a] = (orc_real)node * c->dx - xp[a];
        I[a] = node + c->ghost;
    }
}

void orc_p2g(const orc_config* c, int64_t N, double dt,
             const orc_real* x, const orc_real* v, const orc_real* C, const orc_real* S,
             orc_real* gm, orc_real* gp)
{
    orc_p2g_ex(c, N, dt, x, v, C, S, gm, gp, NULL);
}

/* As orc_p2g; gq (may be NULL) also receives the nodal momentum without the
 * internal force, sum phi m_p (v_p + C_p (x_i - x_p)), from which the grid
 * velocity before the update, v_i^n = gq / m_i, is formed for FLIP. */
void orc_p2g_ex(const orc_config* c, int64_t N, double dt,
                const orc_real* x, const orc_real* v, const orc_real* C, const orc_real* S,
                orc_real* gm, orc_real* gp, orc_real* gq)
{
    int d = dimv(c);
    int32_t dims[3];
    int64_t NN = orc_node_dims(c, dims);
    memset(gm, 0, sizeof(orc_real) * (size_t)NN);
    memset(gp, 0, sizeof(orc_real) * (size_t)(NN * d));
    if (gq) memset(gq, 0, sizeof(orc_real) * (size_t)(NN * d));
    int kz_max = (d == 3) ? 3 : 1;
    for (int64_t p = 0; p < N; ++p) {
        stencil st;
        make_stencil(c, N, x, p, &st);
        orc_real xp[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
            xp[a] = x[a * N + p];
            vp[a] = v[a * N + p];
        }
        for (int k2 = 0; k2 < kz_max; ++k2)
            for (int k1 = 0; k1 < 3; ++k1)
                for (int k0 = 0; k0 < 3; ++k0) {
                    int k[3] = {k0, k1, k2};
                    orc_real phi, grad[3], dpos[3];
                    int32_t I[3];
                    stencil_node(c, xp, &st, k, &phi, grad, dpos, I);
                    int64_t li = node_lin(dims, I);
                    gm[li] += phi * c->mass;
                    for (int a = 0; a < d; ++a) {
                        orc_real aff = 0.0;   /* (C_p (x_i - x_p))_a */
                        orc_real frc = 0.0;   /* (S_p grad phi)_a */
                        for (int b = 0; b < d; ++b) {
                            aff += C[(a * d + b) * N + p] * dpos[b];
                            frc += S[(a * d + b) * N + p] * grad[b];
                        }
                        gp[a * NN + li] += phi * c->mass * (vp[a] + aff) - dt * frc;
                        if (gq) gq[a * NN + li] += phi * c->mass * (vp[a] + aff);
                    }
                }
    }
}

/* ------------------------------------------------------------------ */
/* Grid update and walls (Sec. 2.2 grid update; Sec. 5.3 friction)     */
/* ------------------------------------------------------------------ */

/* Coulomb / slip / stick on one node for the wall with outward normal nrm. */
static void wall_apply(int d, int mode, orc_real mu, const double nrm[3], orc_real vel[3])
{
    orc_real vn = 0.0;
    for (int a = 0; a < d; ++a)
        vn += vel[a] * nrm[a];
    if (!(RE(vn) > 0.0))
        return; /* separating or resting: no constraint */
    orc_real vt[3] = {0, 0, 0}, vtn2 = 0.0;
    for (int a = 0; a < d; ++a) {
        vt[a] = vel[a] - vn * nrm[a];
        vtn2 += vt[a] * vt[a];
    }
    if (mode == ORC_WALL_SLIP) {
        for (int a = 0; a < d; ++a)
            vel[a] = vt[a];
        return;
    }
    if (mode == ORC_WALL_STICK) {
        for (int a = 0; a < d; ++a)
            vel[a] = 0.0;
        return;
    }
    /* Coulomb with a resting wall (v_cm = 0): remove the normal part and
     * reduce the tangential speed by mu * v_n, stopping if it would reverse. */
    orc_real vtn = SQRT(vtn2);
    if (RE(vtn) <= RE(mu * vn)) {
        for (int a = 0; a < d; ++a)
            vel[a] = 0.0;
    } else {
        orc_real scale = 1.0 - mu * vn / vtn;
        for (int a = 0; a < d; ++a)
            vel[a] = vt[a] * scale;
    }
}

/* Resting rigid obstacles (Sec. 4.2.1): frictionless contact removes the
 * normal velocity of a node at the interface, v = v~ - (v~ . n) n.
 * Readings: a node is at the interface of obstacle box [lo, hi] when it lies
 * in the closed box; n is the normal of the nearest face that is not on the
 * domain boundary (ties: the first in the order x-, x+, y-, y+, z-, z+);
 * as for the walls and in the contact method the paper cites, the
 * correction acts only while the node moves into the obstacle; obstacles
 * are applied after the walls, in their order. */
void orc_obstacles(const orc_config* c, const int32_t I[3], orc_real vel[3])
{
    int d = dimv(c);
    for (int o = 0; o < c->n_obstacles; ++o) {
        double xi[3] = {0, 0, 0};
        int inside = 1;
        for (int a = 0; a < d; ++a) {
            xi[a] = (double)(I[a] - c->ghost) * c->dx;
            if (xi[a] < c->obst_lo[o][a] || xi[a] > c->obst_hi[o][a]) inside = 0;
        }
        if (!inside) continue;
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
        if (best_a < 0) continue;
        /* n points into the obstacle: +e_a through its lower face */
        orc_real vn = best_side == 0 ? vel[best_a] : -vel[best_a];
        if (RE(vn) > 0.0) vel[best_a] = 0.0;
    }
}

void orc_grid_update(const orc_config* c, double dt, const orc_real* floor_mu,
                     const orc_real* gm, const orc_real* gp, orc_real* gv)
{
    int d = dimv(c);
    int32_t dims[3];
    int64_t NN = orc_node_dims(c, dims);
    int fl = d - 1; /* floor = minus face of the last axis */
    for (int32_t Iz = 0; Iz < dims[2]; ++Iz)
        for (int32_t Iy = 0; Iy < dims[1]; ++Iy)
            for (int32_t Ix = 0; Ix < dims[0]; ++Ix) {
                int32_t I[3] = {Ix, Iy, Iz};
                int64_t li = node_lin(dims, I);
                orc_real vel[3] = {0, 0, 0};
                if (RE(gm[li]) > 0.0) {
                    for (int a = 0; a < d; ++a)
                        vel[a] = gp[a * NN + li] / gm[li] + dt * c->gravity[a];
                }
                for (int a = 0; a < d; ++a) {
                    int32_t i = I[a] - c->ghost; /* physical node index */
                    for (int side = 0; side < 2; ++side) {
                        int face = 2 * a + side;
                        int beyond = side == 0 ? (i <= 0) : (i >= c->n[a]);
                        if (!beyond)
                            continue;
                        double nrm[3] = {0, 0, 0};
                        nrm[a] = side == 0 ? -1.0 : 1.0;
                        orc_real mu = c->wall_mu[face];
                        if (floor_mu && a == fl && side == 0) {
                            int64_t fi = (d == 3) ? ((int64_t)Iy * dims[0] + Ix) : Ix;
                            mu = floor_mu[fi];
                        }
                        wall_apply(d, c->wall_mode[face], mu, nrm, vel);
                    }
                }
                if (RE(gm[li]) > 0.0) orc_obstacles(c, I, vel);
                for (int a = 0; a < d; ++a)
                    gv[a * NN + li] = vel[a];
            }
}

/* ------------------------------------------------------------------ */
/* G2P (Sec. 2.2 PIC velocity, position, velocity gradient; App. B)   */
/* ------------------------------------------------------------------ */

void orc_g2p(const orc_config* c, int64_t N, double dt, const orc_real* gv,
             orc_real* x, orc_real* v, orc_real* C, orc_real* L)
{
    orc_g2p_ex(c, N, dt, gv, NULL, x, v, C, L);
}

/* G2P with the configured transfer (Sec. 2.2 G2P; App. B):
 *   APIC  v' = sum phi v_i,  C' = (4/h^2) sum phi v_i (x_i - x_p)^T
 *   PIC   v' = sum phi v_i,  C' = 0
 *   TPIC  v' = sum phi v_i,  C' = grad v (the next P2G's affine matrix)
 *   FLIP  v' = sum phi v_i + alpha (v_p - sum phi v_i^n), C' = 0; alpha = 1
 *         is FLIP (v_p + dt sum phi a_i), alpha = 0 PIC, between: the blend.
 * Reading: the grid acceleration of FLIP is (v_i^{n+1} - v_i^n) / dt with
 * v_i^{n+1} after the walls and obstacles and v_i^n = gq / m (gvo), so the
 * boundary conditions reach FLIP particles too.  Every transfer moves the
 * particle with the interpolated new grid velocity. */
void orc_g2p_ex(const orc_config* c, int64_t N, double dt, const orc_real* gv, const orc_real* gvo,
                orc_real* x, orc_real* v, orc_real* C, orc_real* L)
{
    int d = dimv(c);
    int32_t dims[3];
    int64_t NN = orc_node_dims(c, dims);
    double Dinv = 4.0 / (c->dx * c->dx);
    int kz_max = (d == 3) ? 3 : 1;
    for (int64_t p = 0; p < N; ++p) {
        stencil st;
        make_stencil(c, N, x, p, &st);
        orc_real xp[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a)
            xp[a] = x[a * N + p];
        orc_real vn[3] = {0, 0, 0}, vo[3] = {0, 0, 0}, Bm[3][3] = {{0}}, Lm[3][3] = {{0}};
        int flip = c->transfer == ORC_FLIP && gvo;
        for (int k2 = 0; k2 < kz_max; ++k2)
            for (int k1 = 0; k1 < 3; ++k1)
                for (int k0 = 0; k0 < 3; ++k0) {
                    int k[3] = {k0, k1, k2};
                    orc_real phi, grad[3], dpos[3];
                    int32_t I[3];
                    stencil_node(c, xp, &st, k, &phi, grad, dpos, I);
                    int64_t li = node_lin(dims, I);
                    for (int a = 0; a < d; ++a) {
                        orc_real vi = gv[a * NN + li];
                        vn[a] += phi * vi;
                        if (flip) vo[a] += phi * gvo[a * NN + li];
                        for (int b = 0; b < d; ++b) {
                            Bm[a][b] += phi * vi * dpos[b];
                            Lm[a][b] += vi * grad[b];
                        }
                    }
                }
        for (int a = 0; a < d; ++a) {
            orc_real vnew = vn[a];
            if (flip) vnew = vn[a] + c->flip_alpha * (v[a * N + p] - vo[a]);
            v[a * N + p] = vnew;
            orc_real xn = xp[a] + dt * vn[a];
            double hi = (double)c->n[a] * c->dx;
            if (RE(xn) < 0.0) xn = 0.0;
            if (RE(xn) > hi) xn = hi;
            x[a * N + p] = xn;
            for (int b = 0; b < d; ++b) {
                orc_real cab;
                switch (c->transfer) {
                case ORC_APIC: cab = Dinv * Bm[a][b]; break;
                case ORC_TPIC: cab = Lm[a][b]; break;
                default: cab = 0.0; break;     /* PIC, FLIP: no affine part */
                }
                C[(a * d + b) * N + p] = cab;
                L[(a * d + b) * N + p] = Lm[a][b];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Small dense linear algebra                                           */
/* ------------------------------------------------------------------ */

static void matmul(int d, const orc_real A[3][3], const orc_real B[3][3], orc_real R[3][3])
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            orc_real s = 0.0;
            for (int k = 0; k < d; ++k)
                s += A[i][k] * B[k][j];
            R[i][j] = s;
        }
}

static orc_real det(int d, const orc_real A[3][3])
{
    if (d == 2)
        return A[0][0] * A[1][1] - A[0][1] * A[1][0];
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Cyclic Jacobi eigen-decomposition of a symmetric d x d matrix A:
 * A = V diag(ev) V^T, iterated until the off-diagonal part is negligible:
 * below 1e-15 of the matrix norm (a few units of rounding of the diagonal;
 * a smaller bound is below what rounding lets the rotations reach, and then
 * every call runs out its sweep budget). */
void orc_sym_eig(int d, const orc_real Ain[9], orc_real ev[3], orc_real Vout[9])
{
    orc_real A[3][3], V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[i][j] = (i < d && j < d) ? Ain[i * d + j] : 0.0;
            V[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        orc_real off = 0.0, tot = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                tot += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (RE(off) <= 1e-30 * RE(tot) || RE(off) == 0.0)
            break;
        for (int p = 0; p < d - 1; ++p)
            for (int q = p + 1; q < d; ++q) {
                if (RE(A[p][q]) == 0.0)
                    continue;
                orc_real theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                orc_real t = (RE(theta) >= 0.0 ? 1.0 : -1.0) / (ABS(theta) + SQRT(theta * theta + 1.0));
                orc_real cs = 1.0 / SQRT(t * t + 1.0), sn = t * cs;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int k = 0; k < d; ++k) {
                    orc_real akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < d; ++k) {
                    orc_real apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < d; ++k) {
                    orc_real vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq;
                    V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i)
        ev[i] = (i < d) ? A[i][i] : 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            Vout[i * d + j] = V[i][j];
}

/* ------------------------------------------------------------------ */
/* Constitutive models                                                  */
/* ------------------------------------------------------------------ */

/* Tait form of the weakly compressible EOS; gamma = 1 with K = rho0 c^2
 * is eq:eos of Sec. 2.3 written in J = rho0/rho. */
orc_real orc_fluid_pressure(const orc_config* c, orc_real J)
{
    return (c->bulk / c->gamma) * (POW(1.0 / J, c->gamma) - 1.0);
}

double orc_cone_alpha(const orc_config* c)
{
    double s = sin(c->phi_deg * M_PI / 180.0);
    double q_phi = 6.0 * s / (sqrt(3.0) * (3.0 + s)); /* App. A */
    return sqrt(2.0) / 3.0 * q_phi;
}

/* Hencky-strain return mapping onto the Drucker-Prager cone.
 * Ftr: trial elastic deformation gradient (d x d, row-major).
 * Outputs the returned elastic F, the Kirchhoff stress tau and the case
 * (0 apex, 1 elastic, 2 cone).  elastic_only forces the elastic case. */
int orc_hencky_return(const orc_config* c, int elastic_only, const orc_real Ftr[9],
                      orc_real Fe[9], orc_real tau[9], orc_real* dgamma)
{
    int d = c->dim;
    double E = c->youngs, nu = c->poisson;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    orc_real F[3][3] = {{0}}, b[9] = {0};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            F[i][j] = Ftr[i * d + j];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            orc_real s = 0.0;
            for (int k = 0; k < d; ++k)
                s += F[i][k] * F[j][k];
            b[i * d + j] = s;
        }
    orc_real ev[3], U[9];
    orc_sym_eig(d, b, ev, U);
    orc_real eps[3] = {0, 0, 0}, sv[3] = {1, 1, 1}, tr = 0.0;
    for (int i = 0; i < d; ++i) {
        sv[i] = SQRT(ev[i]);
        eps[i] = LOG(sv[i]);
        tr += eps[i];
    }
    orc_real dev[3] = {0, 0, 0}, devn = 0.0;
    for (int i = 0; i < d; ++i) {
        dev[i] = eps[i] - tr / d;
        devn += dev[i] * dev[i];
    }
    devn = SQRT(devn);
    orc_real H[3] = {0, 0, 0};
    int cas;
    orc_real dg = 0.0;
    orc_real en2 = 0.0;
    for (int i = 0; i < d; ++i) en2 += eps[i] * eps[i];
    if (elastic_only || RE(en2) <= ORC_EPS_ELASTIC * ORC_EPS_ELASTIC) {
        /* elastic material, or a strain below the elastic band (reading:
         * the return is not differentiable at zero strain, so the case is
         * fixed there instead of being left to rounding) */
        cas = 1;
        for (int i = 0; i < d; ++i) H[i] = eps[i];
    } else if (RE(tr) > 0.0) {
        cas = 0; /* apex: stress free */
        orc_real en = 0.0;
        for (int i = 0; i < d; ++i) en += eps[i] * eps[i];
        dg = SQRT(en);
    } else {
        double alpha = orc_cone_alpha(c);
        dg = devn + (d * lam + 2.0 * mu) / (2.0 * mu) * alpha * tr;
        if (RE(dg) <= 0.0) {
            cas = 1;
            dg = 0.0;
            for (int i = 0; i < d; ++i) H[i] = eps[i];
        } else {
            cas = 2;
            for (int i = 0; i < d; ++i) H[i] = eps[i] - dg * dev[i] / devn;
        }
    }
    orc_real trH = 0.0;
    for (int i = 0; i < d; ++i) trH += H[i];
    /* Fe = U diag(EXP(H)/s) U^T Ftr ; tau = U diag(2 mu H + lam trH) U^T */
    orc_real M[3][3] = {{0}}, T[3][3] = {{0}};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            orc_real m = 0.0, t = 0.0;
            for (int k = 0; k < d; ++k) {
                m += U[i * d + k] * (EXP(H[k]) / sv[k]) * U[j * d + k];
                t += U[i * d + k] * (2.0 * mu * H[k] + lam * trH) * U[j * d + k];
            }
            M[i][j] = m;
            T[i][j] = t;
        }
    orc_real R[3][3];
    if (cas == 1) {
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                R[i][j] = F[i][j];
    } else {
        matmul(d, M, F, R);
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            Fe[i * d + j] = R[i][j];
            tau[i * d + j] = T[i][j];
        }
    if (dgamma) *dgamma = dg;
    return cas;
}

/* Newtonian fluid (Sec. 2.3 eq:stress_strain): Kirchhoff stress
 * tau = J sigma with sigma = -p I + 2 mu (d - tr(d)/3 I), d = (L + L^T)/2.
 * Readings: the printed increment Delta d stands where the rate d is meant
 * (a stress needs the rate, units Pa = Pa s * 1/s); in 2-D the 3 is the
 * dimension, so that the viscous stress stays traceless there too. */
void orc_fluid_stress(const orc_config* c, orc_real J, const orc_real L[9], orc_real tau[9])
{
    int d = dimv(c);
    orc_real pr = orc_fluid_pressure(c, J);
    orc_real trd = 0.0;
    for (int a = 0; a < d; ++a) trd += L[a * d + a];
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            orc_real rate = 0.5 * (L[a * d + b] + L[b * d + a]);
            orc_real sig = 2.0 * c->viscosity * rate;
            if (a == b) sig += -pr - 2.0 * c->viscosity * trd / d;
            tau[a * d + b] = J * sig;
        }
}

/* Hypoelastic Drucker-Prager with the Jaumann rate, shear yielding and a
 * tension cutoff (Sec. 2.3 eq:dp_stress; App. A steps (1)-(5)).  sigma is
 * the Cauchy stress (d x d, row-major), updated in place; L the velocity
 * gradient of the step, (L)_ab = d v_a / d x_b.  Returns the zone: 1
 * elastic, 2 shear failure, 3 tensile failure; *deps_eq (may be NULL) the
 * equivalent plastic strain increment.
 *   (1) Delta d = dt (L + L^T)/2, Delta w = dt (L - L^T)/2,
 *       sigma^R_ij = sigma_ij + sigma_ik Dw_jk + sigma_jk Dw_ik,
 *       trial = sigma^R + lam tr(Delta d) I + 2 G Delta d;
 *   (2) sigma_m = tr/d, tau = SQRT(s:s / 2);
 *   (3) f^s = tau - k_phi + q_phi sigma_m, f^t = sigma_m - sigma^t,
 *       h = tau - tau^P - alpha^P (sigma_m - sigma^t);
 *   (4) zone II: dl = f^s / (G + K q_phi q_psi), sigma_m -= K q_psi dl,
 *       tau = k_phi - q_phi sigma_m, s scaled to tau;
 *   (5) zone III: sigma_m = sigma^t, s kept.
 * Readings (no value or rule in the paper): in 2-D the mean is tr/2 and
 * K = lam + G (the 2-D bulk modulus), the paper's 3 being the dimension;
 * a shear return that ends beyond the cutoff (sigma_m > sigma^t, reached
 * only from the corner branch h > 0, f^t >= 0) is taken to the corner
 * (sigma^t, tau^P); a trial stress of Frobenius norm at or below 1e-6 E is
 * elastic whatever its zone (the zones meet at zero stress, where a body at
 * rest sits). */
int orc_dp_jaumann(const orc_config* c, double dt, const orc_real L[9], orc_real sigma[9],
                   orc_real* deps_eq)
{
    int d = dimv(c);
    double E = c->youngs, nu = c->poisson;
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double G = E / (2.0 * (1.0 + nu));
    double K = lam + 2.0 * G / d;
    double sp = sin(c->phi_deg * M_PI / 180.0), cp = cos(c->phi_deg * M_PI / 180.0);
    double ss = sin(c->psi_deg * M_PI / 180.0);
    double q_phi = 6.0 * sp / (sqrt(3.0) * (3.0 + sp));
    double k_phi = 6.0 * c->cohesion * cp / (sqrt(3.0) * (3.0 + sp));
    double q_psi = 6.0 * ss / (sqrt(3.0) * (3.0 + ss));
    double st = c->tension;
    double tauP = k_phi - q_phi * st;
    double alphaP = sqrt(1.0 + q_phi * q_phi) - q_phi;

    orc_real Dd[3][3] = {{0}}, Dw[3][3] = {{0}}, S0[3][3] = {{0}};
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            Dd[a][b] = 0.5 * dt * (L[a * d + b] + L[b * d + a]);
            Dw[a][b] = 0.5 * dt * (L[a * d + b] - L[b * d + a]);
            S0[a][b] = sigma[a * d + b];
        }
    orc_real trD = 0.0;
    for (int a = 0; a < d; ++a) trD += Dd[a][a];
    orc_real Tr[3][3];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            orc_real r = S0[i][j];
            for (int k = 0; k < d; ++k) r += S0[i][k] * Dw[j][k] + S0[j][k] * Dw[i][k];
            Tr[i][j] = r + 2.0 * G * Dd[i][j] + (i == j ? lam * trD : 0.0);
        }
    orc_real sm = 0.0;
    for (int a = 0; a < d; ++a) sm += Tr[a][a];
    sm /= d;
    orc_real s[3][3], ss2 = 0.0, nrm2 = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            s[i][j] = Tr[i][j] - (i == j ? sm : 0.0);
            ss2 += s[i][j] * s[i][j];
            nrm2 += Tr[i][j] * Tr[i][j];
        }
    orc_real tau = SQRT(0.5 * ss2);
    orc_real fs = tau - k_phi + q_phi * sm;
    orc_real ft = sm - st;
    orc_real h = tau - tauP - alphaP * (sm - st);
    int zone;
    if (RE(SQRT(nrm2)) <= 1e-6 * E) zone = 1;
    else if (RE(ft) < 0.0) zone = RE(fs) <= 0.0 ? 1 : 2;
    else zone = RE(h) > 0.0 ? 2 : 3;
    orc_real sm_n = sm, scale = 1.0, de = 0.0;
    if (zone == 2) {
        orc_real dl = fs / (G + K * q_phi * q_psi);
        sm_n = sm - K * q_psi * dl;
        orc_real tau_n = k_phi - q_phi * sm_n;
        if (RE(sm_n) > st) {          /* beyond the cutoff: the corner */
            sm_n = st;
            tau_n = tauP;
        }
        scale = RE(tau) > 0.0 ? tau_n / tau : 0.0;
        de = dl * sqrt(1.0 / 3.0 + 2.0 / 9.0 * q_psi * q_psi);
    } else if (zone == 3) {
        sm_n = st;
        de = sqrt(2.0) / 3.0 * (sm - st) / K;
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            sigma[i * d + j] = scale * s[i][j] + (i == j ? sm_n : 0.0);
    if (deps_eq) *deps_eq = de;
    return zone;
}

/* Kinematics (F or J update with the velocity gradient L) followed by the
 * stress of the material; S = V0 * tau (Kirchhoff stress times initial
 * volume, equal to V_p sigma_p).  For the hypoelastic Drucker-Prager
 * material the carried stress is S = V_p sigma = V0 J sigma: the Cauchy
 * stress of the step is S / (V0 J) with the J before the update.
 * eps (may be NULL) accumulates the equivalent plastic strain: for the
 * hypoelastic material App. A's increment (zone II: dl sqrt(1/3 + 2/9
 * q_psi^2), zone III: sqrt(2)/3 (sigma_m - sigma^t)/K); for the Hencky
 * return (reading) the von Mises equivalent sqrt(2/3) |dE_p| of the plastic
 * log-strain increment dE_p = eps - H, whose norm is the return's dgamma. */
void orc_constitutive(const orc_config* c, int64_t N, double dt, const orc_real* L,
                      orc_real* F, orc_real* J, orc_real* S, orc_real* eps)
{
    int d = dimv(c);
    for (int64_t p = 0; p < N; ++p) {
        orc_real M[3][3] = {{0}}; /* I + dt L */
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                M[a][b] = (a == b ? 1.0 : 0.0) + dt * L[(a * d + b) * N + p];
        orc_real tau[3][3] = {{0}};
        if (c->material == ORC_FLUID) {
            orc_real Jn = J[p] * det(d, M);
            J[p] = Jn;
            orc_real Lp[9], tu[9];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) Lp[a * d + b] = L[(a * d + b) * N + p];
            orc_fluid_stress(c, Jn, Lp, tu);
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) tau[a][b] = tu[a * d + b];
        } else if (c->material == ORC_DP_JAUMANN) {
            orc_real Jo = J[p], Jn = Jo * det(d, M);
            orc_real Lp[9], sg[9];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    Lp[a * d + b] = L[(a * d + b) * N + p];
                    sg[a * d + b] = S[(a * d + b) * N + p] / (c->vol0 * Jo);
                }
            orc_real de = 0.0;
            orc_dp_jaumann(c, dt, Lp, sg, &de);
            if (eps) eps[p] += de;
            J[p] = Jn;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) tau[a][b] = Jn * sg[a * d + b];
        } else {
            orc_real Fo[3][3] = {{0}}, Ft[3][3];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b)
                    Fo[a][b] = F[(a * d + b) * N + p];
            matmul(d, M, Fo, Ft);
            orc_real ftr[9], fe[9], tu[9];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b)
                    ftr[a * d + b] = Ft[a][b];
            orc_real dg = 0.0;
            orc_hencky_return(c, c->material == ORC_HENCKY_ELASTIC, ftr, fe, tu, &dg);
            if (eps) eps[p] += sqrt(2.0 / 3.0) * dg;
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) {
                    F[(a * d + b) * N + p] = fe[a * d + b];
                    tau[a][b] = tu[a * d + b];
                }
        }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                S[(a * d + b) * N + p] = c->vol0 * tau[a][b];
    }
}

/* ------------------------------------------------------------------ */
/* One full step: sort, P2G, grid update with walls, G2P, constitutive  */
/* ------------------------------------------------------------------ */

int orc_step(const orc_config* c, int64_t N, double dt, const orc_real* floor_mu,
             orc_real* x, orc_real* v, orc_real* C, orc_real* F, orc_real* J, orc_real* S,
             int32_t* pid, int32_t* perm_out, int32_t* key_out,
             orc_real* grid_m_out, orc_real* grid_v_out, orc_real* eps)
{
    int d = dimv(c);
    int32_t dims[3];
    int64_t NN = orc_node_dims(c, dims);
    size_t NP = (size_t)(N > 0 ? N : 1);
    int32_t* key = (int32_t*)malloc(sizeof(int32_t) * NP);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * NP);
    int32_t* itmp = (int32_t*)malloc(sizeof(int32_t) * NP);
    orc_real* tmp = (orc_real*)malloc(sizeof(orc_real) * NP);
    orc_real* L = (orc_real*)malloc(sizeof(orc_real) * NP * (size_t)(d * d));
    orc_real* gm = (orc_real*)malloc(sizeof(orc_real) * (size_t)NN);
    orc_real* gp = (orc_real*)malloc(sizeof(orc_real) * (size_t)(NN * d));
    orc_real* gv = (orc_real*)malloc(sizeof(orc_real) * (size_t)(NN * d));
    if (!key || !perm || !itmp || !tmp || !L || !gm || !gp || !gv) {
        free(key); free(perm); free(itmp); free(tmp); free(L); free(gm); free(gp); free(gv);
        return -1;
    }

    orc_cell_keys(c, N, x, key);
    orc_sort_perm(N, key, orc_cells_per_tile(c), perm);
    gather_d(N, d, x, perm, tmp);
    gather_d(N, d, v, perm, tmp);
    gather_d(N, d * d, C, perm, tmp);
    gather_d(N, d * d, S, perm, tmp);
    if (c->material == ORC_FLUID || c->material == ORC_DP_JAUMANN)
        gather_d(N, 1, J, perm, tmp);
    if (c->material != ORC_FLUID)
        gather_d(N, d * d, F, perm, tmp);
    if (eps)
        gather_d(N, 1, eps, perm, tmp);
    gather_i(N, pid, perm, itmp);
    if (perm_out) memcpy(perm_out, perm, sizeof(int32_t) * (size_t)N);
    if (key_out) memcpy(key_out, key, sizeof(int32_t) * (size_t)N);

    /* FLIP needs the grid velocity before the update, v_i^n = gq / m_i */
    orc_real* gq = NULL;
    if (c->transfer == ORC_FLIP) {
        gq = (orc_real*)malloc(sizeof(orc_real) * (size_t)(NN * d));
        if (!gq) {
            free(key); free(perm); free(itmp); free(tmp); free(L); free(gm); free(gp); free(gv);
            return -1;
        }
    }
    orc_p2g_ex(c, N, dt, x, v, C, S, gm, gp, gq);
    orc_grid_update(c, dt, floor_mu, gm, gp, gv);
    if (gq)
        for (int64_t i = 0; i < NN; ++i)
            for (int a = 0; a < d; ++a)
                gq[a * NN + i] = RE(gm[i]) > 0.0 ? gq[a * NN + i] / gm[i] : 0.0;
    if (grid_m_out) memcpy(grid_m_out, gm, sizeof(orc_real) * (size_t)NN);
    if (grid_v_out) memcpy(grid_v_out, gv, sizeof(orc_real) * (size_t)(NN * d));
    orc_g2p_ex(c, N, dt, gv, gq, x, v, C, L);
    orc_constitutive(c, N, dt, L, F, J, S, eps);

    free(key); free(perm); free(itmp); free(tmp); free(L); free(gm); free(gp); free(gv); free(gq);
    return 0;
}
