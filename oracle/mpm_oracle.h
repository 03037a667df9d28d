/*
 * Oracle (test infrastructure only): binary64 reference MPM step.
 * Declarations for mpm_oracle.c and mpm_oracle_adjoint.c.  Nothing in the
 * HIP library includes this header.
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H
#include <stdint.h>

/* Number type of the particle and grid data: binary64, or complex binary64
 * in the complex-step build of the forward step (ORC_COMPLEX_STEP), which
 * only the adjoint's checks use. */
#ifdef ORC_COMPLEX_STEP
#include <complex.h>
#undef I /* the oracle names node indices I */
typedef double _Complex orc_real;
#else
typedef double orc_real;
#endif

enum { ORC_FLUID = 0, ORC_DP_HENCKY = 1, ORC_HENCKY_ELASTIC = 2, ORC_DP_JAUMANN = 3 };
enum { ORC_WALL_SLIP = 0, ORC_WALL_STICK = 1, ORC_WALL_COULOMB = 2 };
/* grid-to-particle transfer (Sec. 2.2 G2P; App. B) */
enum { ORC_APIC = 0, ORC_PIC = 1, ORC_FLIP = 2, ORC_TPIC = 3 };
#define ORC_MAX_OBSTACLES 4

/* Hencky strain magnitude |eps|_F at or below which the Drucker-Prager
 * return takes the elastic case whatever the sign of tr(eps) (a reading:
 * the apex is not differentiable, so at rounding-level strain the case is
 * fixed by this rule rather than by the rounding of tr(eps)). */
#define ORC_EPS_ELASTIC 1e-6

typedef struct orc_config {
    int32_t dim;          /* 2 or 3 */
    int32_t n[3];         /* cells per axis */
    int32_t ghost;        /* ghost node layers per side */
    int32_t tile;         /* tile edge in cells, for the cell key */
    int32_t material;     /* ORC_FLUID / ORC_DP_HENCKY / ORC_HENCKY_ELASTIC */
    int32_t key_f32;      /* 1: stencil base computed in binary32 */
    int32_t wall_mode[6]; /* faces x-, x+, y-, y+, z-, z+ */
    double dx;
    double gravity[3];
    double wall_mu[6];
    double rho0, bulk, gamma;          /* fluid */
    double youngs, poisson, phi_deg;   /* sand */
    double vol0, mass;                 /* per particle */
    int32_t transfer;     /* ORC_APIC / ORC_PIC / ORC_FLIP / ORC_TPIC */
    int32_t n_obstacles;  /* resting rigid boxes, <= ORC_MAX_OBSTACLES */
    double flip_alpha;    /* FLIP share of the FLIP/PIC blend (1 = FLIP) */
    double viscosity;     /* fluid: dynamic viscosity mu (eq:stress_strain) */
    double psi_deg, cohesion, tension;   /* App. A: dilation angle, c, sigma^t */
    double obst_lo[ORC_MAX_OBSTACLES][3], obst_hi[ORC_MAX_OBSTACLES][3];
} orc_config;

orc_real orc_phibar(orc_real xi);
orc_real orc_dphibar(orc_real xi);
void orc_stencil_1d(orc_real x, double h, int key_f32, int32_t* base, orc_real w[3], orc_real dw[3]);
int64_t orc_node_dims(const orc_config* c, int32_t dims[3]);
int64_t orc_num_keys(const orc_config* c);
int64_t orc_key_of_base(const orc_config* c, const int32_t B[3]);
void orc_cell_keys(const orc_config* c, int64_t N, const orc_real* x, int32_t* key);
int32_t orc_cells_per_tile(const orc_config* c);
void orc_sort_perm(int64_t N, const int32_t* key, int32_t cpt, int32_t* perm);
void orc_p2g(const orc_config* c, int64_t N, double dt, const orc_real* x, const orc_real* v,
             const orc_real* C, const orc_real* S, orc_real* gm, orc_real* gp);
void orc_p2g_ex(const orc_config* c, int64_t N, double dt, const orc_real* x, const orc_real* v,
                const orc_real* C, const orc_real* S, orc_real* gm, orc_real* gp, orc_real* gq);
void orc_grid_update(const orc_config* c, double dt, const orc_real* floor_mu,
                     const orc_real* gm, const orc_real* gp, orc_real* gv);
void orc_g2p(const orc_config* c, int64_t N, double dt, const orc_real* gv,
             orc_real* x, orc_real* v, orc_real* C, orc_real* L);
void orc_g2p_ex(const orc_config* c, int64_t N, double dt, const orc_real* gv, const orc_real* gvo,
                orc_real* x, orc_real* v, orc_real* C, orc_real* L);
void orc_obstacles(const orc_config* c, const int32_t I[3], orc_real vel[3]);
int orc_dp_jaumann(const orc_config* c, double dt, const orc_real L[9], orc_real sigma[9],
                   orc_real* deps_eq);
void orc_fluid_stress(const orc_config* c, orc_real J, const orc_real L[9], orc_real tau[9]);
void orc_sym_eig(int d, const orc_real A[9], orc_real ev[3], orc_real V[9]);
orc_real orc_fluid_pressure(const orc_config* c, orc_real J);
double orc_cone_alpha(const orc_config* c);
int orc_hencky_return(const orc_config* c, int elastic_only, const orc_real Ftr[9],
                      orc_real Fe[9], orc_real tau[9], orc_real* dgamma);
void orc_constitutive(const orc_config* c, int64_t N, double dt, const orc_real* L,
                      orc_real* F, orc_real* J, orc_real* S, orc_real* eps);
int orc_step(const orc_config* c, int64_t N, double dt, const orc_real* floor_mu,
             orc_real* x, orc_real* v, orc_real* C, orc_real* F, orc_real* J, orc_real* S,
             int32_t* pid, int32_t* perm_out, int32_t* key_out,
             orc_real* grid_m_out, orc_real* grid_v_out, orc_real* eps);

#endif
