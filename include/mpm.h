/*
 * mpm.h -- C-ABI of the MI355X explicit MPM solver (gfx950, HIP).
 *
 * The calls follow the paper's statement of the problem (Du & He,
 * "JAX-MPM", arXiv 2507.04192):
 *   - a state S = {x, v, F, rho} advanced by one map per step,
 *     S^{t+1} = Phi(S^t; alpha), Phi = G2P o GU o P2G      (Sec. 3.1, eq:mapping)
 *   - P2G, grid update and G2P as in Sec. 2.2, APIC as in App. B,
 *     stress update last (USL, Sec. 2.2 remark)
 *   - extraction operators Q_l (Lagrangian tracer, Eulerian box mean) and the
 *     masked least-squares loss                           (Sec. 3.2, eq:inverse_loss)
 *   - dL/dalpha by a reverse sweep over checkpointed segments (Sec. 3.1
 *     eq:dzda; Sec. 3.3 checkpointing and segmentation)
 *   - parameters alpha as an initial velocity field or a per-node floor
 *     friction, optionally produced by a small network   (Sec. 3.2, eq:nn_apprx)
 *
 * Conventions (all calls):
 *   - Return value: MPM_OK (0) or a negative mpm_status.  No exception crosses
 *     the ABI.  mpm_last_error() gives a message for the last failure.
 *   - Pointers are device pointers on the context's device unless the name
 *     starts with host_.  Floating-point buffers use the context's precision
 *     (binary32 or binary64) unless stated otherwise.
 *   - Particle arrays are structure-of-arrays, component-major: component a
 *     of particle p at [a*n + p]; matrix entry (a,b) at [(a*dim+b)*n + p].
 *   - The caller owns every buffer it passes in; the context keeps only
 *     views into the workspace bound by mpm_bind_workspace().
 *   - Work is queued on the stream given to mpm_create() and is asynchronous
 *     unless the call says it synchronizes.
 */
#ifndef MPM_H
#define MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mpm_status {
    MPM_OK = 0,
    MPM_EINVAL = -1,      /* bad argument or configuration */
    MPM_ENOMEM = -2,      /* workspace missing or too small */
    MPM_EHIP = -3,        /* a HIP runtime call or launch failed */
    MPM_ENONFINITE = -4,  /* a particle's state became NaN or Inf */
    MPM_EDOMAIN = -5,     /* a particle moved more than one cell in a step (CFL) */
    MPM_ESTATE = -6,      /* call made in the wrong order */
    MPM_ECONVERGE = -7    /* binary64: a particle's eigen-solve (Hencky return) did not converge */
} mpm_status;

enum { MPM_F32 = 0, MPM_F64 = 1 };

/* Materials (Sec. 2.3):
 *  FLUID_TAIT     weakly compressible fluid, p = (K/gamma)((1/J)^gamma - 1);
 *                 gamma = 1 with K = rho0 c^2 is eq:eos
 *  DP_HENCKY      Drucker-Prager sand: Hencky strain of F_e, radial return onto
 *                 the cone with slope (sqrt2/3) q_phi (q_phi of App. A),
 *                 stress-free apex for tr(eps) > 0; elastic whenever
 *                 |eps|_F <= 1e-6 (the case at rounding-level strain)
 *  HENCKY_ELASTIC the same elastic law without the return (checks only)
 *  DP_JAUMANN     the paper's own Drucker-Prager (Sec. 2.3 eq:dp_stress; App. A):
 *                 hypoelastic Cauchy stress rotated with the Jaumann rate,
 *                 Delta d = dt (L + L^T)/2, Delta w = dt (L - L^T)/2, trial
 *                 stress by the isotropic elastic tensor, then zones I (elastic),
 *                 II (shear return along the plastic potential of dilation
 *                 angle psi) and III (tension cutoff sigma_m = sigma^t); a shear
 *                 return that ends beyond the cutoff stops at the corner
 *                 (sigma^t, tau^P); a trial stress of Frobenius norm <= 1e-6 E is
 *                 elastic.  Carries J = J det(I + dt L) and the stress cache
 *                 V0 J sigma.  In 2-D the mean stress is tr/2 and K = lam + G.
 * A FLUID_TAIT material with viscosity > 0 adds the Newtonian stress of
 * Sec. 2.3 eq:stress_strain, 2 mu (d - tr(d)/dim I) with the rate
 * d = (L + L^T)/2, and then carries the full symmetric stress. */
enum { MPM_FLUID_TAIT = 0, MPM_DP_HENCKY = 1, MPM_HENCKY_ELASTIC = 2, MPM_DP_JAUMANN = 3 };

/* Grid-to-particle transfer (Sec. 2.2 G2P; App. B), v_i the grid velocity
 * after the update and walls, x_i - x_p the node offset:
 *  APIC  v' = sum phi v_i,  C' = (4/h^2) sum phi v_i (x_i - x_p)^T
 *  PIC   v' = sum phi v_i,  C' = 0
 *  TPIC  v' = sum phi v_i,  C' = sum v_i (grad phi)^T (the velocity gradient)
 *  FLIP  v' = sum phi v_i + flip_alpha (v_p - sum phi v_i^n), C' = 0, with
 *        v_i^n = (P2G momentum without the internal force) / m_i: flip_alpha
 *        = 1 is FLIP, 0 is PIC, between them the FLIP/PIC blend.
 * Every transfer moves the particle with the interpolated new velocity,
 * x' = x + dt sum phi v_i, and P2G uses the carried C as the affine term. */
enum { MPM_XFER_APIC = 0, MPM_XFER_PIC = 1, MPM_XFER_FLIP = 2, MPM_XFER_TPIC = 3 };

/* Resting rigid obstacles (Sec. 4.2.1, frictionless contact): axis-aligned
 * boxes [lo, hi].  After the walls, a node with mass inside the closed box
 * whose velocity points into the obstacle through its nearest face (faces
 * on the domain boundary excluded; ties: the first face in the order x-,
 * x+, y-, y+, z-, z+) loses that normal component, v = v - (v.n) n.
 * Obstacles apply in their order. */
#define MPM_MAX_OBSTACLES 4

/* Wall behaviour on a face (Sec. 2.2 ghost cells; Sec. 5.3 eq:coulomb_friction
 * with a resting wall).  Applies to nodes on or beyond the wall plane and only
 * while the node velocity points into the wall. */
enum { MPM_WALL_SLIP = 0, MPM_WALL_STICK = 1, MPM_WALL_COULOMB = 2 };

/* Particle fields for mpm_read_state / mpm_write_state. */
enum {
    MPM_FIELD_X = 0,      /* position, dim comps */
    MPM_FIELD_V = 1,      /* velocity, dim comps */
    MPM_FIELD_C = 2,      /* APIC affine matrix, dim*dim comps */
    MPM_FIELD_F = 3,      /* elastic deformation gradient, dim*dim (Hencky materials) */
    MPM_FIELD_FMI = 4,    /* F - I, dim*dim (Hencky materials); stored form, exact */
    MPM_FIELD_J = 5,      /* volume ratio J = rho0/rho, 1 comp (fluid, DP_JAUMANN) */
    MPM_FIELD_JM1 = 6,    /* J - 1, 1 comp (fluid, DP_JAUMANN); stored form, exact */
    MPM_FIELD_STRESS = 7, /* V0 * Kirchhoff stress = V_p sigma_p, dim*dim */
    MPM_FIELD_PID = 8,    /* original particle index, int32 */
    MPM_FIELD_EPS_EQ = 9  /* equivalent plastic strain accumulated by mpm_step, 1 comp
                           * (needs track_eps_eq): DP_JAUMANN App. A's increment
                           * (zone II: dl sqrt(1/3 + 2/9 q_psi^2); zone III:
                           * sqrt(2)/3 (sigma_m - sigma^t)/K), DP_HENCKY the von Mises
                           * equivalent sqrt(2/3)|dE_p| of the plastic log-strain
                           * increment (|dE_p| = the return's dgamma); 0 for the other
                           * materials.  Starts at 0 at mpm_init_particles. */
};
enum { MPM_ORDER_MEMORY = 0, MPM_ORDER_PID = 1 };

/* Grid fields for mpm_read_grid: last step's nodal mass and nodal velocity
 * after the grid update and walls, on the dense node box of
 * (n[a] + 1 + 2*ghost) nodes per axis, x fastest. */
enum { MPM_GRID_MASS = 0, MPM_GRID_VEL = 1 };

#define MPM_MAX_TAPE_SEGMENTS 64

typedef struct mpm_config {
    int32_t dim;           /* 2 or 3 */
    int32_t precision;     /* MPM_F32 or MPM_F64 */
    int32_t n[3];          /* cells per axis; domain is [0, n[a]*dx] */
    int32_t ghost;         /* ghost node layers per side, >= 1 */
    int32_t tile;          /* tile edge in cells: 4 (3D) or 8 (2D); 0 = default */
    int32_t material;      /* MPM_FLUID_TAIT, MPM_DP_HENCKY, MPM_HENCKY_ELASTIC, MPM_DP_JAUMANN */
    int32_t wall_mode[6];  /* faces x-, x+, y-, y+, z-, z+ */
    int32_t keep_grid;     /* 1: keep nodal mass for mpm_read_grid */
    double dx;             /* grid spacing */
    double gravity[3];     /* body force per unit mass */
    double wall_mu[6];     /* Coulomb coefficient per face */
    double rho0, bulk, gamma;         /* fluid: reference density, K, gamma */
    double youngs, poisson, phi_deg;  /* sand: E, nu, friction angle */
    /* added physics; the zero defaults keep the APIC step without them */
    int32_t transfer;      /* MPM_XFER_APIC (0), _PIC, _FLIP or _TPIC */
    int32_t n_obstacles;   /* resting rigid boxes in obst_lo/hi, 0..MPM_MAX_OBSTACLES */
    double flip_alpha;     /* FLIP share of the FLIP/PIC blend, in [0, 1] (FLIP only) */
    double viscosity;      /* FLUID_TAIT: dynamic viscosity mu >= 0 (Pa s) */
    double psi_deg;        /* DP_JAUMANN: dilation angle, 0 <= psi <= phi */
    double cohesion;       /* DP_JAUMANN: c >= 0 */
    double tension;        /* DP_JAUMANN: tensile strength sigma^t, <= k_phi / q_phi (the apex) */
    double obst_lo[MPM_MAX_OBSTACLES][3], obst_hi[MPM_MAX_OBSTACLES][3];   /* lo < hi per used axis */
    /* memory for speed in a forward-plus-adjoint rollout: the number of
     * trailing segments kept on the tape, whose steps the backward sweep
     * does not recompute (0 or 1: the last segment; at most the number of
     * segments and MPM_MAX_TAPE_SEGMENTS; each costs ckpt_every + 1 states
     * and ckpt_every grid records of workspace) */
    int32_t tape_segments;
    /* 1: carry the equivalent plastic strain (MPM_FIELD_EPS_EQ) through
     * mpm_step: two more scalars per particle of workspace, and G2P reads and
     * writes one more per step (plastic materials); mpm_forward_loss then
     * returns EINVAL.  0: not carried. */
    int32_t track_eps_eq;
} mpm_config;

typedef struct mpm_ctx mpm_ctx;

/* Validates cfg and creates a context on the current device, bound to
 * hip_stream (a hipStream_t; NULL = default stream).  Allocates no device
 * memory.  *out receives the context; EINVAL on a bad configuration,
 * including a grid whose tile count times 64 reaches 2^31 (cell keys are
 * int32). */
int mpm_create(const mpm_config* cfg, void* hip_stream, mpm_ctx** out);

/* Device bytes needed for n_particles and, if tape_steps > 0, for a
 * forward-plus-adjoint rollout of tape_steps steps checkpointed every
 * ckpt_every steps (Sec. 3.3: memory O(N_t / n) per segment): one state per
 * checkpoint, a tape of ckpt_every + 1 states, and a grid tape holding each
 * step of a segment's sort and nodal mass and velocities. */
int mpm_workspace_bytes(const mpm_config* cfg, int64_t n_particles, int32_t tape_steps,
                        int32_t ckpt_every, size_t* bytes);

/* Binds caller-owned device memory (>= mpm_workspace_bytes for the same
 * arguments, 256-byte aligned).  The memory must stay valid until
 * mpm_destroy.  Clears the grid.  ENOMEM if too small. */
int mpm_bind_workspace(mpm_ctx* ctx, void* dev_ptr, size_t bytes, int64_t n_particles,
                       int32_t tape_steps, int32_t ckpt_every);

/* Sets n particles (n <= the bound capacity) from x[dim][n] and v[dim][n]
 * (device, context precision), with C = 0, F = I (sand) or J = 1 (fluid),
 * zero stress cache and pid = 0..n-1; mass and vol0 per particle (eq:semi:
 * m_p and V_p at rest).  Computes the first cell keys. */
int mpm_init_particles(mpm_ctx* ctx, int64_t n, const void* x, const void* v,
                       double vol0, double mass);

/* Per-node Coulomb coefficient of the floor (minus face of the last axis),
 * overriding wall_mu for that face: count = n[0]+1+2G values in 2D,
 * (n[0]+1+2G)*(n[1]+1+2G) in 3D, x fastest (device, context precision).
 * mu = NULL restores the face constant.  The pointer is kept, not copied. */
int mpm_set_floor_mu(mpm_ctx* ctx, const void* mu, int64_t count);

/* Advances n steps of size dt (Sec. 2.2, USL): per step the particles are
 * sorted by cell key, P2G, grid update with gravity and walls, G2P with the
 * velocity gradient, then the constitutive update.  Asynchronous; data errors
 * (non-finite state, a particle moving more than one cell in a step) are
 * latched and reported by mpm_sync_status. */
int mpm_step(mpm_ctx* ctx, int32_t n, double dt);

/* Synchronizes the stream and returns the latched data status: MPM_OK,
 * MPM_ENONFINITE (checked first), MPM_EDOMAIN (|v| dt > dx on an axis:
 * the step violates the CFL condition) or MPM_ECONVERGE (binary64 only: the
 * Jacobi eigen-solve that the Hencky return falls back to for large strains
 * ran out of sweeps before its off-diagonal part was negligible); *bad_pid
 * (may be NULL) gets the smallest offending pid or -1.  Clears the latch. */
int mpm_sync_status(mpm_ctx* ctx, int64_t* bad_pid);

/* Copies a particle field to dst (device; int32 for PID), in memory order or
 * in pid order.  EINVAL for a field the material does not carry. */
int mpm_read_state(mpm_ctx* ctx, int32_t field, int32_t order, void* dst);

/* Overwrites a particle field from src (same layout as mpm_read_state).
 * Writing X recomputes the cell keys.  PID cannot be written. */
int mpm_write_state(mpm_ctx* ctx, int32_t field, int32_t order, const void* src);

/* Last step's grid field (see MPM_GRID_*), dense node box, device dst.
 * Nodes outside the last step's active tiles (no particle near them) read
 * as zero.  MASS needs keep_grid = 1. */
int mpm_read_grid(mpm_ctx* ctx, int32_t which, void* dst);

/* Last step's sort: perm[s] = memory slot, before the step, of the particle
 * now in slot s; key[s] = cell key of the current positions (used by the
 * next step).  int32 device arrays of n; either may be NULL. */
int mpm_read_sort(mpm_ctx* ctx, void* perm, void* key);

/* Observations for the inverse problem (Sec. 3.2, eq:inverse_loss):
 *   L = sum over frames t and indices l of m_{l,t} |Q_l(z^t) - z^obs_{l,t}|^2
 * with the Lagrangian operator Q_l(z) = z of tracked particle l and the
 * Eulerian operator Q_l = mean of z over the particles inside box l.  An
 * empty box contributes nothing; box membership is held fixed when
 * differentiating.  Device arrays are kept (not copied) until the next call
 * and must stay valid; host arrays are copied. */
#define MPM_MAX_BOXES 64
typedef struct mpm_obs {
    int32_t n_frames;
    const int32_t* host_frames;  /* steps after which the state is observed: ascending, >= 1 */
    int32_t n_tracers;           /* Lagrangian operator; 0 for none */
    const int32_t* tracer_pid;   /* device int32[n_tracers]: particle ids */
    int32_t lag_field;           /* MPM_FIELD_X or MPM_FIELD_V */
    const void* lag_target;      /* device [n_frames][dim][n_tracers], context precision */
    const void* lag_mask;        /* device [n_frames][n_tracers] 0/1 weights, or NULL for all 1 */
    int32_t n_boxes;             /* Eulerian operator; 0 for none, at most MPM_MAX_BOXES */
    const double* host_box_lo;   /* host [n_boxes][dim]: box is [lo, hi) on every axis */
    const double* host_box_hi;
    int32_t eul_field;           /* MPM_FIELD_X or MPM_FIELD_V */
    const void* eul_target;      /* device [n_frames][dim][n_boxes] */
    const void* eul_mask;        /* device [n_frames][n_boxes] or NULL */
} mpm_obs;

int mpm_set_observations(mpm_ctx* ctx, const mpm_obs* obs);

/* Runs n_steps steps from the current state (the parameters alpha being the
 * current particle velocities and the floor friction set by
 * mpm_set_floor_mu), storing a checkpoint every ckpt_every steps (the values
 * given to mpm_bind_workspace; n_steps <= its tape_steps) and accumulating
 * the loss of the observations in binary64.  The last segment runs directly
 * on the tape, so that the first mpm_backward after it need not recompute
 * it.  Synchronizes; *host_loss gets the loss.  The state, sort and grid
 * afterwards are those after n_steps, as after mpm_step(n_steps).  The
 * reverse sweep covers every material (the viscous fluid included), resting
 * obstacles and every transfer (FLIP's also through the grid velocity
 * before the update, which the tape then records).  EINVAL with
 * track_eps_eq set (the equivalent plastic strain is a forward diagnostic,
 * carried by mpm_step only). */
int mpm_forward_loss(mpm_ctx* ctx, int32_t n_steps, double dt, double* host_loss);

/* Gradient of the last mpm_forward_loss by the hand-written reverse sweep:
 * each segment between checkpoints is recomputed (the grid of each step is
 * kept on the grid tape), then every step is reversed (constitutive update,
 * G2P, walls, grid, P2G, sort).  May be called again for the same rollout:
 * node adjoints are summed with atomics, so repeated calls agree to rounding,
 * not bit for bit.  grad_v0
 * (device [dim][n], pid order) receives dL/dv of the rollout's initial
 * state, grad_mu (device, floor layout of mpm_set_floor_mu) dL/dmu per floor
 * node (zero without a friction field).  Either may be NULL.  Synchronizes.
 * ESTATE without a preceding mpm_forward_loss. */
int mpm_backward(mpm_ctx* ctx, void* grad_v0, void* grad_mu);

/* Learned parameter field alpha(x) ~ N_theta(x) (Sec. 3.2, eq:nn_apprx): a
 * small MLP on the matrix cores.  Layers l = 0..n_layers-1 map width[l] to
 * width[l+1]; hidden layers use hidden_act (tanh by default, or ReLU as in
 * the velocity-profile network of Sec. 5.2); the output layer applies out_act and
 * then y = out_shift + out_scale * act(z).  Inputs are first mapped
 * feature-wise to in_scale[k] * x_k + in_shift[k].  math selects the MFMA
 * operand type: BF16 operands with FP32 accumulation, or FP32 operands.
 * Parameters are FP32: for each layer W_l (width[l+1] x width[l],
 * row-major) then b_l, layers concatenated.  x is [width[0]][n] and y, dy
 * are [width[n_layers]][n] (component-major, like particle fields); cache
 * and work are scratch of mpm_mlp_cache_floats(n) floats each.  These calls
 * need no solver context; they queue work on hip_stream. */
#define MPM_MLP_MAX_LAYERS 4
#define MPM_MLP_MAX_IN 4
enum { MPM_ACT_NONE = 0, MPM_ACT_SIGMOID = 1 };
enum { MPM_HIDDEN_TANH = 0, MPM_HIDDEN_RELU = 1 };
enum { MPM_MLP_BF16 = 0, MPM_MLP_F32 = 1 };
typedef struct mpm_mlp {
    int32_t n_layers;                       /* 1..MPM_MLP_MAX_LAYERS */
    int32_t width[MPM_MLP_MAX_LAYERS + 1];  /* each in [1, 128]; width[0] <= MPM_MLP_MAX_IN */
    int32_t out_act;                        /* MPM_ACT_NONE or MPM_ACT_SIGMOID */
    int32_t math;                           /* MPM_MLP_BF16 or MPM_MLP_F32 */
    float out_scale, out_shift;
    float in_scale[MPM_MLP_MAX_IN], in_shift[MPM_MLP_MAX_IN];
    int32_t hidden_act;                     /* MPM_HIDDEN_TANH (0) or MPM_HIDDEN_RELU */
} mpm_mlp;

/* Number of parameters, or -1 for an invalid description. */
int64_t mpm_mlp_num_params(const mpm_mlp* net);
/* Floats of the activation cache (and of the backward work buffer) for n samples. */
int64_t mpm_mlp_cache_floats(const mpm_mlp* net, int64_t n);
/* y = N_theta(x) for n samples; fills cache for mpm_mlp_backward. */
int mpm_mlp_forward(const mpm_mlp* net, void* hip_stream, const float* params, int64_t n, const float* x,
                    float* y, float* cache);
/* dparams = gradient of sum(dy * y) with respect to the parameters (the
 * buffer is overwritten), using the cache of the matching forward call. */
int mpm_mlp_backward(const mpm_mlp* net, void* hip_stream, const float* params, int64_t n, const float* x,
                     const float* cache, const float* dy, float* work, float* dparams);
/* The same backward pass for callers that cannot allocate device memory
 * (code under HIP graph capture, tight training or serving loops, harnesses
 * that forbid hipMalloc): the work buffer is a static device array of
 * MPM_MLP_SCRATCH_FLOATS floats (32 MiB) that every GPU the library runs on
 * holds until the process ends, looked up on the first call on a device.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  EINVAL (message in mpm_last_error(NULL)) when
 * mpm_mlp_cache_floats(net, n) exceeds MPM_MLP_SCRATCH_FLOATS.  Every call
 * on one GPU shares that GPU's array (it keeps the last call's contents;
 * the kernels write every entry they read): calls that overlap on one GPU,
 * on different streams or from different threads, race. */
#define MPM_MLP_SCRATCH_FLOATS (8 * 1024 * 1024)
int mpm_mlp_backward_noalloc(const mpm_mlp* net, void* hip_stream, const float* params, int64_t n,
                             const float* x, const float* cache, const float* dy, float* dparams);
/* One Adam update (Kingma & Ba) of n parameters in place; step >= 1 counts
 * updates; m and v are the moment buffers (start at zero). */
int mpm_adam_step(void* hip_stream, int64_t n, float* params, const float* grad, float* m, float* v,
                  int32_t step, double lr, double beta1, double beta2, double eps);

/* Plain parametric field, the fallback of the learned one (Sec. 3.2,
 * parameter forms): nc components piecewise constant on an nx x ny cell grid
 * over [lo, hi) of the first two coordinates (host_lo, host_hi: 2 doubles);
 * points outside take the nearest cell.  x: [>=2][n] FP32 positions,
 * table: [nc][ny][nx] FP32, out/dout: [nc][n].  gather: out = table(cell(x));
 * scatter: dtable (overwritten) = per-cell sums of dout (the adjoint). */
int mpm_cell_field_gather(void* hip_stream, int32_t nc, int32_t nx, int32_t ny, const double* host_lo,
                          const double* host_hi, int64_t n, const float* x, const float* table, float* out);
int mpm_cell_field_scatter(void* hip_stream, int32_t nc, int32_t nx, int32_t ny, const double* host_lo,
                           const double* host_hi, int64_t n, const float* x, const float* dout, float* dtable);

/* The extraction operators of the set observations applied to the current
 * state: lag_q [dim][n_tracers] (tracer values) and eul_q [dim][n_boxes]
 * (box means; zero for an empty box), device, context precision; either may
 * be NULL.  Used to record synthetic observations from a ground-truth run. */
int mpm_extract(mpm_ctx* ctx, void* lag_q, void* eul_q);

/* Per-kernel-class timing of mpm_step, mpm_forward_loss and mpm_backward:
 * with profiling on, HIP events are recorded on the context's stream between
 * the kernel classes below, and mpm_profile_read (synchronizes) returns, per
 * class, the summed event time in milliseconds and the number of launches
 * since the last read, then resets.  Arrays hold MPM_PROF_N entries (host
 * memory).  In the backward sweep the recomputed forward kernels count in
 * their own classes (the key pass of a recomputed step counts as SCAN), the
 * reverse kernels in the *_ADJ classes. */
enum { MPM_PROF_SCAN = 0, MPM_PROF_BUCKET = 1, MPM_PROF_P2G = 2, MPM_PROF_GRID = 3, MPM_PROF_G2P = 4,
       MPM_PROF_G2P_ADJ = 5, MPM_PROF_GRID_ADJ = 6, MPM_PROF_P2G_ADJ = 7, MPM_PROF_N = 8 };
int mpm_profile_enable(mpm_ctx* ctx, int on);
int mpm_profile_read(mpm_ctx* ctx, double* host_ms, int64_t* host_launches);

/* Number of particles currently set. */
int64_t mpm_num_particles(const mpm_ctx* ctx);

/* Message of the last failure on ctx (or, when ctx is NULL, of the last
 * failed call without a context on this thread: mpm_create,
 * mpm_mlp_backward_noalloc).  Valid until the next such call. */
const char* mpm_last_error(const mpm_ctx* ctx);

/* Frees the context (not the caller's workspace).  Synchronizes the stream. */
int mpm_destroy(mpm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MPM_H */
