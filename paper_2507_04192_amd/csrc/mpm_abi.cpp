// C-ABI of the solver: configuration checks, workspace layout and binding,
// and dispatch to the per-precision operation tables.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <string>

#include <algorithm>
#include "mpm_runtime.hpp"

using namespace mpm;

// Message of the last failure of a call without a context (mpm_create,
// mpm_workspace_bytes, the context-free calls): a fixed buffer, so that
// recording it allocates nothing.
static thread_local char g_global_error[256] = "";

void mpm::set_global_error(const char* msg)
{
    strncpy(g_global_error, msg ? msg : "", sizeof(g_global_error) - 1);
    g_global_error[sizeof(g_global_error) - 1] = 0;
}

namespace {

int nsym_of(int dim) { return dim * (dim + 1) / 2; }

// Kernel material of a configuration: an inviscid fluid carries one
// isotropic stress value, a viscous one the full symmetric stress.
int kernel_mat(const mpm_config& c)
{
    switch (c.material) {
    case MPM_FLUID_TAIT: return c.viscosity > 0.0 ? MAT_VFLUID : MAT_FLUID;
    case MPM_DP_HENCKY: return MAT_SAND;
    case MPM_HENCKY_ELASTIC: return MAT_ELASTIC;
    default: return MAT_JAUMANN;
    }
}

int nsc_of(const mpm_config& c)
{
    int D = c.dim, m = kernel_mat(c);
    return 2 * D + D * D + (mat_has_F(m) ? D * D : 1) + (mat_iso_stress(m) ? 1 : nsym_of(D));
}

bool is_flip(const mpm_config& c) { return c.transfer == MPM_XFER_FLIP; }

int check_config(const mpm_config* c, std::string& why)
{
    if (!c) { why = "config is NULL"; return MPM_EINVAL; }
    if (c->dim != 2 && c->dim != 3) { why = "dim must be 2 or 3"; return MPM_EINVAL; }
    if (c->precision != MPM_F32 && c->precision != MPM_F64) { why = "precision must be MPM_F32 or MPM_F64"; return MPM_EINVAL; }
    for (int a = 0; a < c->dim; ++a)
        if (c->n[a] < 1 || c->n[a] > 8192) { why = "cells per axis must be in [1, 8192]"; return MPM_EINVAL; }
    if (c->ghost < 1 || c->ghost > 8) { why = "ghost must be in [1, 8]"; return MPM_EINVAL; }
    {
        // cell keys are int32: tile count * 64 cells must stay below 2^31
        long long tiles = 1;
        int T = c->dim == 3 ? 4 : 8;
        for (int a = 0; a < c->dim; ++a) tiles *= ((long long)c->n[a] + 2 * c->ghost + 1 + T - 1) / T;
        if (tiles * 64 >= (1ll << 31)) { why = "grid too large for 32-bit cell keys (tiles * 64 >= 2^31)"; return MPM_EINVAL; }
    }
    int want_tile = c->dim == 3 ? 4 : 8;
    if (c->tile != 0 && c->tile != want_tile) { why = "tile must be 4 in 3D and 8 in 2D (64 cells per tile)"; return MPM_EINVAL; }
    if (!(c->dx > 0.0) || !isfinite(c->dx)) { why = "dx must be positive"; return MPM_EINVAL; }
    if (c->material < MPM_FLUID_TAIT || c->material > MPM_DP_JAUMANN) { why = "unknown material"; return MPM_EINVAL; }
    if (c->transfer < MPM_XFER_APIC || c->transfer > MPM_XFER_TPIC) { why = "unknown transfer"; return MPM_EINVAL; }
    if (c->transfer == MPM_XFER_FLIP && !(c->flip_alpha >= 0.0 && c->flip_alpha <= 1.0)) {
        why = "flip_alpha must be in [0, 1]";
        return MPM_EINVAL;
    }
    if (c->n_obstacles < 0 || c->n_obstacles > MPM_MAX_OBSTACLES) { why = "n_obstacles must be in [0, 4]"; return MPM_EINVAL; }
    if (c->tape_segments < 0 || c->tape_segments > MPM_MAX_TAPE_SEGMENTS) { why = "tape_segments must be in [0, 64]"; return MPM_EINVAL; }
    if (c->track_eps_eq != 0 && c->track_eps_eq != 1) { why = "track_eps_eq must be 0 or 1"; return MPM_EINVAL; }
    for (int o = 0; o < c->n_obstacles; ++o)
        for (int a = 0; a < c->dim; ++a)
            if (!isfinite(c->obst_lo[o][a]) || !isfinite(c->obst_hi[o][a]) || !(c->obst_lo[o][a] < c->obst_hi[o][a])) {
                why = "obstacle boxes need finite lo < hi on every axis";
                return MPM_EINVAL;
            }
    if (!(c->viscosity >= 0.0) || !isfinite(c->viscosity)) { why = "viscosity must be finite and >= 0"; return MPM_EINVAL; }
    if (c->viscosity > 0.0 && c->material != MPM_FLUID_TAIT) { why = "viscosity applies to the fluid only"; return MPM_EINVAL; }
    for (int f = 0; f < 6; ++f) {
        if (c->wall_mode[f] < MPM_WALL_SLIP || c->wall_mode[f] > MPM_WALL_COULOMB) { why = "unknown wall mode"; return MPM_EINVAL; }
        if (!(c->wall_mu[f] >= 0.0)) { why = "wall friction must be >= 0"; return MPM_EINVAL; }
    }
    for (int a = 0; a < 3; ++a)
        if (!isfinite(c->gravity[a])) { why = "gravity must be finite"; return MPM_EINVAL; }
    if (c->material == MPM_FLUID_TAIT) {
        if (!(c->rho0 > 0.0) || !(c->bulk > 0.0) || !(c->gamma > 0.0)) { why = "fluid needs rho0, bulk, gamma > 0"; return MPM_EINVAL; }
    } else {
        if (!(c->youngs > 0.0) || !(c->poisson > -1.0 && c->poisson < 0.5)) { why = "need E > 0 and -1 < nu < 0.5"; return MPM_EINVAL; }
        if (!(c->phi_deg >= 0.0 && c->phi_deg < 90.0)) { why = "friction angle must be in [0, 90)"; return MPM_EINVAL; }
    }
    if (c->material == MPM_DP_JAUMANN) {
        if (!(c->psi_deg >= 0.0 && c->psi_deg <= c->phi_deg)) { why = "dilation angle must be in [0, phi]"; return MPM_EINVAL; }
        if (!(c->cohesion >= 0.0) || !isfinite(c->cohesion)) { why = "cohesion must be finite and >= 0"; return MPM_EINVAL; }
        double sp = sin(c->phi_deg * M_PI / 180.0), cp = cos(c->phi_deg * M_PI / 180.0);
        double q_phi = 6.0 * sp / (sqrt(3.0) * (3.0 + sp)), k_phi = 6.0 * c->cohesion * cp / (sqrt(3.0) * (3.0 + sp));
        // the cutoff lies at or below the apex of the cone (sigma_m = k_phi / q_phi)
        bool ok = isfinite(c->tension) && (q_phi > 0.0 ? c->tension * q_phi <= k_phi : true);
        if (!ok) { why = "tension must be finite and at or below the apex k_phi / q_phi"; return MPM_EINVAL; }
    }
    return MPM_OK;
}

Geo make_geo(const mpm_config& c)
{
    Geo g{};
    g.dim = c.dim;
    g.T = c.dim == 3 ? 4 : 8;
    g.G = c.ghost;
    g.NN = 1;
    g.ntiles = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < c.dim) {
            g.n[a] = c.n[a];
            g.bmax[a] = c.n[a] + 2 * c.ghost;
            int span = c.n[a] + 2 * c.ghost + 1;
            g.ntile[a] = (span + g.T - 1) / g.T;
            g.nd[a] = g.ntile[a] * g.T + 2;
            g.box[a] = c.n[a] + 1 + 2 * c.ghost;
        } else {
            g.n[a] = 1;
            g.bmax[a] = 0;
            g.ntile[a] = 1;
            g.nd[a] = 1;
            g.box[a] = 1;
        }
        g.NN *= g.nd[a];
        g.ntiles *= g.ntile[a];
    }
    return g;
}

struct Layout {
    size_t st[2], pid[2], eps[2], key, perm, tmp, tmpk, count, tile_off, tile_slot, active, part, meta, status;
    size_t part_grid, gv, gmass, gvo;
    size_t inv, loss, box_sum, box_cnt, box_coef;
    size_t ckpt, ckpt_pid, tape, tape_pid, adj[2], mid, gtape, amu;
    GridRec grec;
    size_t total;
};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Trailing segments kept on the tape: at least one, at most the rollout's
// segments.
int tape_segs_of(const mpm_config& c, int tape_steps, int ckpt_every)
{
    if (tape_steps < 1 || ckpt_every < 1) return 0;
    int nseg = (tape_steps + ckpt_every - 1) / ckpt_every;
    return std::max(1, std::min(c.tape_segments, nseg));
}

Layout make_layout(const mpm_config& c, const Geo& g, int64_t cap, int tape_steps, int ckpt_every)
{
    Layout L{};
    size_t elem = c.precision == MPM_F64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    size_t ucap = (size_t)(cap > 0 ? cap : 1);
    for (int b = 0; b < 2; ++b) L.st[b] = take((size_t)nsc_of(c) * ucap * elem);
    for (int b = 0; b < 2; ++b) L.pid[b] = take(ucap * 4);
    for (int b = 0; b < 2; ++b) L.eps[b] = c.track_eps_eq ? take(ucap * elem) : 0;
    L.key = take(ucap * 4);
    L.perm = take(ucap * 4);
    L.tmp = take(ucap * 4);
    L.tmpk = take(ucap * 4);
    L.count = take((size_t)g.ntiles * 4);
    L.tile_off = take((size_t)g.ntiles * 4);
    L.tile_slot = take((size_t)g.ntiles * 4);
    L.active = take((size_t)g.ntiles * sizeof(ActiveTile));
    size_t nsb = (size_t)((g.ntiles + kScanChunk - 1) / kScanChunk);
    L.part = take(nsb * 2 * 4);
    L.meta = take(64 * 4);
    L.status = take(64 * 4);
    int nb = c.dim == 3 ? 216 : 100;   // node block of a tile
    // node values per block node: mass and momentum, and for FLIP the
    // momentum without the internal force
    int nv = is_flip(c) ? 2 * c.dim + 1 : c.dim + 1;
    L.part_grid = take((size_t)g.ntiles * nv * nb * elem);
    L.gv = take((size_t)g.NN * c.dim * elem);
    L.gmass = take((size_t)g.NN * elem);
    L.gvo = is_flip(c) ? take((size_t)g.NN * c.dim * elem) : 0;
    L.inv = take(ucap * 4);
    L.loss = take(4 * 8);
    L.box_sum = take(kMaxBoxes * 3 * 8);
    L.box_cnt = take(kMaxBoxes * 4);
    L.box_coef = take(kMaxBoxes * 3 * 8);
    if (tape_steps > 0 && ckpt_every > 0) {
        size_t sb = (size_t)nsc_of(c) * ucap * elem;
        size_t nck = (size_t)((tape_steps + ckpt_every - 1) / ckpt_every);
        size_t nts = (size_t)tape_segs_of(c, tape_steps, ckpt_every);
        L.ckpt = take(nck * sb);
        L.ckpt_pid = take(nck * ucap * 4);
        L.tape = take(nts * (size_t)(ckpt_every + 1) * sb);
        L.tape_pid = take(nts * (size_t)(ckpt_every + 1) * ucap * 4);
        L.adj[0] = take(sb);
        L.adj[1] = take(sb);
        // position and F adjoints (FLIP: and the direct velocity adjoint)
        L.mid = take((size_t)(c.dim + c.dim * c.dim + (is_flip(c) ? c.dim : 0)) * ucap * elem);
        // grid tape: one record per step of a segment
        GridRec& r = L.grec;
        size_t ro = 0;
        auto rtake = [&](size_t bytes) {
            size_t o = ro;
            ro = align_up(ro + bytes);
            return o;
        };
        r.gv = rtake((size_t)g.NN * c.dim * elem);
        r.gvt = rtake((size_t)g.NN * c.dim * elem);
        r.gmass = rtake((size_t)g.NN * elem);
        r.gvo = is_flip(c) ? rtake((size_t)g.NN * c.dim * elem) : 0;   // FLIP: velocity before the update
        r.perm = rtake(ucap * 4);
        r.tile_slot = rtake((size_t)g.ntiles * 4);
        r.active = rtake((size_t)g.ntiles * sizeof(ActiveTile));
        r.meta = rtake(64 * 4);
        r.bytes = ro;
        L.gtape = take(nts * (size_t)ckpt_every * r.bytes);
        size_t nfl = c.dim == 3 ? (size_t)g.box[0] * g.box[1] : (size_t)g.box[0];
        L.amu = take(nfl * 8);
    }
    L.total = off;
    return L;
}

const Ops* pick_ops(const mpm_config& c)
{
    if (c.precision == MPM_F32) return c.dim == 2 ? &ops_f32_2d : &ops_f32_3d;
    return c.dim == 2 ? &ops_f64_2d : &ops_f64_3d;
}

int need_bound(mpm_ctx* c)
{
    if (!c) return MPM_EINVAL;
    if (!c->bound) return set_err(c, MPM_ESTATE, "no workspace bound (call mpm_bind_workspace)");
    return MPM_OK;
}

int need_particles(mpm_ctx* c)
{
    int rc = need_bound(c);
    if (rc) return rc;
    if (!c->has_particles) return set_err(c, MPM_ESTATE, "no particles (call mpm_init_particles)");
    return MPM_OK;
}

}  // namespace

extern "C" {

int mpm_create(const mpm_config* cfg, void* hip_stream, mpm_ctx** out)
{
    if (!out) {
        set_global_error("out is NULL");
        return MPM_EINVAL;
    }
    *out = nullptr;
    std::string why;
    int rc = check_config(cfg, why);
    if (rc) {
        set_global_error(why.c_str());
        return rc;
    }
    mpm_ctx* c = new (std::nothrow) mpm_ctx();
    if (!c) {
        set_global_error("out of host memory");
        return MPM_ENOMEM;
    }
    c->cfg = *cfg;
    c->cfg.tile = cfg->dim == 3 ? 4 : 8;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        set_global_error("hipGetDevice failed");
        delete c;
        return MPM_EHIP;
    }
    c->geo = make_geo(c->cfg);
    c->elem = cfg->precision == MPM_F64 ? 8 : 4;
    c->nsc = nsc_of(c->cfg);
    c->nsym = nsym_of(cfg->dim);
    c->mat = kernel_mat(c->cfg);
    c->xfer = c->cfg.transfer;
    c->ops = pick_ops(c->cfg);
    *out = c;
    return MPM_OK;
}

int mpm_workspace_bytes(const mpm_config* cfg, int64_t n_particles, int32_t tape_steps, int32_t ckpt_every,
                        size_t* bytes)
{
    std::string why;
    int rc = check_config(cfg, why);
    if (rc) {
        set_global_error(why.c_str());
        return rc;
    }
    if (!bytes || n_particles < 0 || n_particles >= (1ll << 31) || tape_steps < 0 || ckpt_every < 0) {
        set_global_error("bad workspace arguments");
        return MPM_EINVAL;
    }
    mpm_config c = *cfg;
    Geo g = make_geo(c);
    *bytes = make_layout(c, g, n_particles, tape_steps, ckpt_every).total;
    return MPM_OK;
}

int mpm_bind_workspace(mpm_ctx* c, void* dev_ptr, size_t bytes, int64_t n_particles, int32_t tape_steps,
                       int32_t ckpt_every)
{
    if (!c) return MPM_EINVAL;
    if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return set_err(c, MPM_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (n_particles < 0 || n_particles >= (1ll << 31) || tape_steps < 0 || ckpt_every < 0)
        return set_err(c, MPM_EINVAL, "bad workspace arguments");
    if (tape_steps > 0 && ckpt_every < 1) return set_err(c, MPM_EINVAL, "a tape needs ckpt_every >= 1");
    Layout L = make_layout(c->cfg, c->geo, n_particles, tape_steps, ckpt_every);
    if (bytes < L.total)
        return set_err(c, MPM_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    char* b = (char*)dev_ptr;
    c->ws = b;
    c->ws_bytes = bytes;
    c->cap = n_particles;
    c->tape_steps = tape_steps;
    c->ckpt_every = ckpt_every;
    c->tape_segs = tape_segs_of(c->cfg, tape_steps, ckpt_every);
    for (int i = 0; i < 2; ++i) {
        c->st[i] = b + L.st[i];
        c->pid[i] = (int32_t*)(b + L.pid[i]);
        c->eps[i] = c->cfg.track_eps_eq ? b + L.eps[i] : nullptr;
    }
    c->key = (int32_t*)(b + L.key);
    c->perm = (int32_t*)(b + L.perm);
    c->tmp = (int32_t*)(b + L.tmp);
    c->tmpk = (int32_t*)(b + L.tmpk);
    c->count = (int32_t*)(b + L.count);
    c->tile_off = (int32_t*)(b + L.tile_off);
    c->tile_slot = (int32_t*)(b + L.tile_slot);
    c->active = (ActiveTile*)(b + L.active);
    c->part = (int32_t*)(b + L.part);
    c->meta = (int32_t*)(b + L.meta);
    c->status = (int32_t*)(b + L.status);
    c->part_grid = b + L.part_grid;
    c->gv = b + L.gv;
    c->gmass = b + L.gmass;
    c->gvo = is_flip(c->cfg) ? b + L.gvo : nullptr;
    c->inv = (int32_t*)(b + L.inv);
    c->loss = (double*)(b + L.loss);
    c->loss_scratch = c->loss + 2;
    c->box_sum = (double*)(b + L.box_sum);
    c->box_cnt = (int32_t*)(b + L.box_cnt);
    c->box_coef = (double*)(b + L.box_coef);
    bool tape = tape_steps > 0 && ckpt_every > 0;
    c->ckpt = tape ? b + L.ckpt : nullptr;
    c->ckpt_pid = tape ? (int32_t*)(b + L.ckpt_pid) : nullptr;
    c->tape = tape ? b + L.tape : nullptr;
    c->tape_pid = tape ? (int32_t*)(b + L.tape_pid) : nullptr;
    c->adj[0] = tape ? b + L.adj[0] : nullptr;
    c->adj[1] = tape ? b + L.adj[1] : nullptr;
    c->mid = tape ? b + L.mid : nullptr;
    c->gtape = tape ? b + L.gtape : nullptr;
    c->grec = L.grec;
    c->amu = tape ? (double*)(b + L.amu) : nullptr;
    c->has_tape = false;
    c->cur = 0;
    c->N = 0;
    c->has_particles = false;
    c->stepped = false;
    c->bound = true;
    return c->ops->clear_grid(c);
}

int mpm_init_particles(mpm_ctx* c, int64_t n, const void* x, const void* v, double vol0, double mass)
{
    int rc = need_bound(c);
    if (rc) return rc;
    if (n < 0 || n > c->cap) return set_err(c, MPM_EINVAL, "particle count exceeds the bound capacity");
    if (n > 0 && (!x || !v)) return set_err(c, MPM_EINVAL, "x and v must be non-null");
    if (!(vol0 > 0.0) || !(mass > 0.0)) return set_err(c, MPM_EINVAL, "vol0 and mass must be positive");
    c->N = n;
    c->mass = mass;
    c->vol0 = vol0;
    c->cur = 0;
    rc = c->ops->init_particles(c, x, v);
    if (rc) return rc;
    c->has_particles = true;
    c->stepped = false;
    return MPM_OK;
}

int mpm_set_floor_mu(mpm_ctx* c, const void* mu, int64_t count)
{
    if (!c) return MPM_EINVAL;
    int64_t want = c->cfg.dim == 3 ? (int64_t)c->geo.box[0] * c->geo.box[1] : c->geo.box[0];
    if (mu && count != want)
        return set_err(c, MPM_EINVAL, "floor friction needs " + std::to_string(want) + " values");
    c->floor_mu = mu;
    return MPM_OK;
}

int mpm_step(mpm_ctx* c, int32_t n, double dt)
{
    int rc = need_particles(c);
    if (rc) return rc;
    if (n < 0) return set_err(c, MPM_EINVAL, "negative step count");
    if (!(dt >= 0.0) || !isfinite(dt)) return set_err(c, MPM_EINVAL, "dt must be finite and >= 0");
    if (n == 0 || c->N == 0) return MPM_OK;
    rc = c->ops->step(c, n, dt);
    if (!rc) c->stepped = true;
    return rc;
}

int mpm_sync_status(mpm_ctx* c, int64_t* bad_pid)
{
    int rc = need_bound(c);
    if (rc) return rc;
    if (bad_pid) *bad_pid = -1;
    rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (rc) return rc;
    int32_t h[4];
    rc = hip_check(c, hipMemcpy(h, c->status, sizeof(h), hipMemcpyDeviceToHost), "status read");
    if (rc) return rc;
    int32_t clear[4] = {0, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    rc = hip_check(c, hipMemcpy(c->status, clear, sizeof(clear), hipMemcpyHostToDevice), "status clear");
    if (rc) return rc;
    if (h[0] & 1) {
        if (bad_pid) *bad_pid = h[1];
        return set_err(c, MPM_ENONFINITE, "non-finite particle state (pid " + std::to_string(h[1]) + ")");
    }
    if (h[0] & 2) {
        if (bad_pid) *bad_pid = h[2];
        return set_err(c, MPM_EDOMAIN, "a particle moved more than one cell in a step (pid " + std::to_string(h[2]) +
                                           "): the time step violates the CFL condition");
    }
    if (h[0] & 4) {
        if (bad_pid) *bad_pid = h[3];
        return set_err(c, MPM_ECONVERGE, "the binary64 eigen-solve of the Hencky return did not converge (pid " +
                                             std::to_string(h[3]) + ")");
    }
    return MPM_OK;
}

int mpm_read_state(mpm_ctx* c, int32_t field, int32_t order, void* dst)
{
    int rc = need_particles(c);
    if (rc) return rc;
    if (!dst && c->N > 0) return set_err(c, MPM_EINVAL, "dst is NULL");
    if (order != MPM_ORDER_MEMORY && order != MPM_ORDER_PID) return set_err(c, MPM_EINVAL, "bad order");
    return c->ops->read_state(c, field, order, dst);
}

int mpm_write_state(mpm_ctx* c, int32_t field, int32_t order, const void* src)
{
    int rc = need_particles(c);
    if (rc) return rc;
    if (!src && c->N > 0) return set_err(c, MPM_EINVAL, "src is NULL");
    if (order != MPM_ORDER_MEMORY && order != MPM_ORDER_PID) return set_err(c, MPM_EINVAL, "bad order");
    return c->ops->write_state(c, field, order, src);
}

int mpm_read_grid(mpm_ctx* c, int32_t which, void* dst)
{
    int rc = need_bound(c);
    if (rc) return rc;
    if (!dst) return set_err(c, MPM_EINVAL, "dst is NULL");
    return c->ops->read_grid(c, which, dst);
}

int mpm_read_sort(mpm_ctx* c, void* perm, void* key)
{
    int rc = need_particles(c);
    if (rc) return rc;
    size_t bytes = sizeof(int32_t) * (size_t)c->N;
    if (perm && c->N > 0) {
        if (!c->stepped) return set_err(c, MPM_ESTATE, "no step taken yet");
        rc = hip_check(c, hipMemcpyAsync(perm, c->perm, bytes, hipMemcpyDeviceToDevice, c->stream), "read perm");
        if (rc) return rc;
    }
    if (key && c->N > 0)
        return hip_check(c, hipMemcpyAsync(key, c->key, bytes, hipMemcpyDeviceToDevice, c->stream), "read key");
    return MPM_OK;
}

int mpm_set_observations(mpm_ctx* c, const mpm_obs* o)
{
    if (!c) return MPM_EINVAL;
    if (!o) return set_err(c, MPM_EINVAL, "obs is NULL");
    if (o->n_frames < 0 || (o->n_frames > 0 && !o->host_frames)) return set_err(c, MPM_EINVAL, "bad frames");
    for (int i = 0; i < o->n_frames; ++i) {
        if (o->host_frames[i] < 1) return set_err(c, MPM_EINVAL, "frames must be >= 1");
        if (i > 0 && o->host_frames[i] <= o->host_frames[i - 1]) return set_err(c, MPM_EINVAL, "frames must ascend");
    }
    if (o->n_tracers < 0 || (o->n_tracers > 0 && (!o->tracer_pid || !o->lag_target)))
        return set_err(c, MPM_EINVAL, "tracers need ids and targets");
    if (o->n_tracers > 0 && o->lag_field != MPM_FIELD_X && o->lag_field != MPM_FIELD_V)
        return set_err(c, MPM_EINVAL, "tracer field must be X or V");
    if (o->n_boxes < 0 || o->n_boxes > MPM_MAX_BOXES) return set_err(c, MPM_EINVAL, "too many boxes");
    if (o->n_boxes > 0 && (!o->host_box_lo || !o->host_box_hi || !o->eul_target))
        return set_err(c, MPM_EINVAL, "boxes need bounds and targets");
    if (o->n_boxes > 0 && o->eul_field != MPM_FIELD_X && o->eul_field != MPM_FIELD_V)
        return set_err(c, MPM_EINVAL, "box field must be X or V");
    c->obs_frames.assign(o->host_frames, o->host_frames + o->n_frames);
    c->obs_ntr = o->n_tracers;
    c->obs_tracer = o->tracer_pid;
    c->obs_lag_field = o->lag_field;
    c->obs_lag_target = o->lag_target;
    c->obs_lag_mask = o->lag_mask;
    c->obs_nbox = o->n_boxes;
    for (int b = 0; b < o->n_boxes; ++b)
        for (int a = 0; a < 3; ++a) {
            c->box_lo[b][a] = a < c->cfg.dim ? o->host_box_lo[b * c->cfg.dim + a] : 0.0;
            c->box_hi[b][a] = a < c->cfg.dim ? o->host_box_hi[b * c->cfg.dim + a] : 0.0;
        }
    c->obs_eul_field = o->eul_field;
    c->obs_eul_target = o->eul_target;
    c->obs_eul_mask = o->eul_mask;
    return MPM_OK;
}

int mpm_forward_loss(mpm_ctx* c, int32_t n_steps, double dt, double* host_loss)
{
    int rc = need_particles(c);
    if (rc) return rc;
    if (!host_loss) return set_err(c, MPM_EINVAL, "host_loss is NULL");
    if (c->cfg.track_eps_eq) return set_err(c, MPM_EINVAL, "track_eps_eq applies to mpm_step only");
    if (!c->ckpt) return set_err(c, MPM_ENOMEM, "no tape: bind the workspace with tape_steps > 0");
    if (n_steps < 1 || n_steps > c->tape_steps) return set_err(c, MPM_EINVAL, "n_steps must be in [1, tape_steps]");
    if (c->N < 1) return set_err(c, MPM_EINVAL, "a rollout needs at least one particle");
    if (!(dt >= 0.0) || !isfinite(dt)) return set_err(c, MPM_EINVAL, "dt must be finite and >= 0");
    c->has_tape = false;
    rc = c->ops->forward_loss(c, n_steps, dt, host_loss);
    if (rc) return rc;
    c->fwd_steps = n_steps;
    c->fwd_dt = dt;
    c->has_tape = true;
    c->stepped = true;
    return MPM_OK;
}

int mpm_backward(mpm_ctx* c, void* grad_v0, void* grad_mu)
{
    int rc = need_particles(c);
    if (rc) return rc;
    if (!c->has_tape) return set_err(c, MPM_ESTATE, "no forward rollout to differentiate (call mpm_forward_loss)");
    return c->ops->backward(c, grad_v0, grad_mu);
}

int mpm_extract(mpm_ctx* c, void* lag_q, void* eul_q)
{
    int rc = need_particles(c);
    if (rc) return rc;
    if (c->N < 1) return set_err(c, MPM_EINVAL, "no particles to observe");
    return c->ops->extract(c, lag_q, eul_q);
}

int mpm_profile_enable(mpm_ctx* c, int on)
{
    if (!c) return MPM_EINVAL;
    c->prof = on != 0;
    return MPM_OK;
}

int mpm_profile_read(mpm_ctx* c, double* host_ms, int64_t* host_launches)
{
    if (!c) return MPM_EINVAL;
    for (int k = 0; k < MPM_PROF_N; ++k) {
        if (host_ms) host_ms[k] = 0.0;
        if (host_launches) host_launches[k] = 0;
    }
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (rc) return rc;
    for (size_t i = 1; i < c->marks.size(); ++i) {
        int cls = c->marks[i].first;
        if (cls < 0 || cls >= MPM_PROF_N) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->marks[i - 1].second, c->marks[i].second) != hipSuccess) continue;
        if (host_ms) host_ms[cls] += ms;
        if (host_launches) host_launches[cls] += 1;
    }
    for (auto& m : c->marks) c->ev_pool.push_back(m.second);
    c->marks.clear();
    return MPM_OK;
}

int64_t mpm_num_particles(const mpm_ctx* c) { return c ? c->N : -1; }

const char* mpm_last_error(const mpm_ctx* c)
{
    if (!c) return g_global_error;
    return c->err.c_str();
}

int mpm_destroy(mpm_ctx* c)
{
    if (!c) return MPM_OK;
    if (c->bound) (void)hipStreamSynchronize(c->stream);
    for (auto& m : c->marks) c->ev_pool.push_back(m.second);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return MPM_OK;
}

}  // extern "C"
