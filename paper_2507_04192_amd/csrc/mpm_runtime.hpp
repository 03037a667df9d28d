// Host runtime state of one solver context and the per-precision operation
// tables.  The context owns no device memory: every device pointer below is
// a view into the caller's workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_types.hpp"

namespace mpm {

constexpr int kBlock = 256;        // threads per workgroup (4 waves)
constexpr int kScanChunk = 2048;   // tiles per scan workgroup
constexpr int kTileWGs = 2048;     // workgroups of the per-tile kernels (8 XCDs x 256)
constexpr int kMaxBoxes = MPM_MAX_BOXES;   // Eulerian observation regions

struct Ops;

// Byte offsets inside one record of the grid tape: what one step's adjoint
// needs from that step's forward pass (nodal velocity after and before the
// walls, nodal mass, the sort permutation and the active-tile list).
struct GridRec {
    size_t gv = 0, gvt = 0, gmass = 0, gvo = 0, perm = 0, tile_slot = 0, active = 0, meta = 0, bytes = 0;
};

}  // namespace mpm

struct mpm_ctx {
    mpm_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    mpm::Geo geo{};
    int elem = 4;                  // bytes per floating-point scalar
    int nsc = 0;                   // scalars per particle per state buffer
    int nsym = 0;                  // stored stress components
    int mat = 0;                   // kernel material (mpm::MAT_*)
    int xfer = 0;                  // transfer (mpm::XF_*)
    const mpm::Ops* ops = nullptr;

    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t cap = 0;               // particle capacity
    int64_t N = 0;                 // particles set
    double mass = 0.0, vol0 = 0.0;  // per particle
    int tape_steps = 0, ckpt_every = 0;
    int tape_segs = 0;             // trailing segments kept on the tape

    void* st[2] = {nullptr, nullptr};        // particle state buffers
    int32_t* pid[2] = {nullptr, nullptr};
    void* eps[2] = {nullptr, nullptr};       // equivalent plastic strain (track_eps_eq), same slots as st
    int cur = 0;
    int32_t* key = nullptr;
    int32_t* perm = nullptr;
    int32_t* tmp = nullptr;
    int32_t* tmpk = nullptr;       // key of each bucketed particle
    int32_t* count = nullptr;
    int32_t* tile_off = nullptr;
    int32_t* tile_slot = nullptr;
    mpm::ActiveTile* active = nullptr;
    int32_t* part = nullptr;
    int32_t* meta = nullptr;       // [0] active tiles, [1] particles sorted
    int32_t* status = nullptr;     // [0] flags, [1] smallest bad pid
    void* part_grid = nullptr;     // per active tile: P2G node block, mass + momentum
    void* gv = nullptr;            // nodal velocity after the grid update [dim]
    void* gmass = nullptr;         // nodal mass kept for read-back
    void* gvo = nullptr;           // FLIP: nodal velocity before the update [dim]
    const void* floor_mu = nullptr;

    // forward-plus-adjoint rollout (mpm_forward_loss / mpm_backward)
    char* ckpt = nullptr;          // checkpoints, one state every ckpt_every steps
    int32_t* ckpt_pid = nullptr;
    char* tape = nullptr;          // states of tape_segs segments (ckpt_every + 1 each)
    int32_t* tape_pid = nullptr;
    char* adj[2] = {nullptr, nullptr};   // adjoint states (same layout as a state)
    void* mid = nullptr;           // per slot: position and F (or J) adjoints between the reverse kernels (FLIP: and the direct velocity adjoint)
    char* gtape = nullptr;         // per step of a segment: the grid and sort it used
    mpm::GridRec grec;
    int32_t* inv = nullptr;        // slot of each pid
    double* amu = nullptr;         // dL/dmu per floor node
    double* loss = nullptr;        // [0] loss of the last forward rollout
    double* loss_scratch = nullptr;
    double* box_sum = nullptr;
    int32_t* box_cnt = nullptr;
    double* box_coef = nullptr;
    int fwd_steps = 0;
    double fwd_dt = 0.0;
    bool has_tape = false;
    int taped = 0;                 // trailing segments of the forward rollout still on the tape

    // observations (mpm_set_observations)
    std::vector<int> obs_frames;
    int obs_ntr = 0;
    const int32_t* obs_tracer = nullptr;
    int obs_lag_field = 0;
    const void* obs_lag_target = nullptr;
    const void* obs_lag_mask = nullptr;
    int obs_nbox = 0;
    double box_lo[MPM_MAX_BOXES][3] = {};
    double box_hi[MPM_MAX_BOXES][3] = {};
    int obs_eul_field = 1;
    const void* obs_eul_target = nullptr;
    const void* obs_eul_mask = nullptr;

    // per-kernel-class timing (mpm_profile_enable)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, hipEvent_t>> marks;

    bool bound = false;
    bool has_particles = false;
    bool stepped = false;
    std::string err;
};

namespace mpm {

struct Ops {
    int (*init_particles)(mpm_ctx*, const void* x, const void* v);
    int (*recompute_keys)(mpm_ctx*);
    int (*clear_grid)(mpm_ctx*);
    int (*step)(mpm_ctx*, int n, double dt);
    int (*read_state)(mpm_ctx*, int field, int order, void* dst);
    int (*write_state)(mpm_ctx*, int field, int order, const void* src);
    int (*read_grid)(mpm_ctx*, int which, void* dst);
    int (*forward_loss)(mpm_ctx*, int n, double dt, double* loss);
    int (*backward)(mpm_ctx*, void* grad_v0, void* grad_mu);
    int (*extract)(mpm_ctx*, void* lag_q, void* eul_q);
};

extern const Ops ops_f32_2d, ops_f32_3d, ops_f64_2d, ops_f64_3d;

// Records an event on the context's stream that closes a span of kernel class
// cls (cls < 0 opens a step).  No-op unless profiling is on.
inline void prof_mark(mpm_ctx* c, int cls)
{
    if (!c->prof || c->marks.size() > 400000) return;
    hipEvent_t e;
    if (!c->ev_pool.empty()) {
        e = c->ev_pool.back();
        c->ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return;
    }
    if (hipEventRecord(e, c->stream) != hipSuccess) {
        c->ev_pool.push_back(e);
        return;
    }
    c->marks.push_back({cls, e});
}

// Records the message of a failed call that has no context (read back by
// mpm_last_error(NULL)); copies into a fixed buffer, allocates nothing.
void set_global_error(const char* msg);

inline int set_err(mpm_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

inline int hip_check(mpm_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MPM_OK;
    return set_err(c, MPM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace mpm
