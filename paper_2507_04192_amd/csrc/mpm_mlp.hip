// Learned field alpha(x) ~ N_theta(x) (Sec. 3.2, eq:nn_apprx): a small MLP
// whose layers run on the matrix cores of gfx950.
//
// Each wave owns 16 samples.  A layer h' = act(h W^T + b) is a 16 x out
// product computed as 16 x 16 output tiles with gfx950's
// v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation, 32-deep K
// steps) or v_mfma_f32_16x16x4_f32 (FP32 operands); activations stay in the
// wave's LDS rows between layers.  Widths are padded to multiples of 16 with
// zeros (the operand functions return zero past the true widths, so a
// 32-deep step may run past the padding).  The weight gradient
// dW = dZ^T H (a reduction over samples) is a split-K MFMA product whose
// partial tiles are added with global atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "../../include/mpm.h"

namespace mpm {
void set_global_error(const char* msg);
}

// Work buffer of mpm_mlp_backward_noalloc (the layer adjoints dZ), a
// file-scope device array: every GPU the library runs on holds one copy
// for the life of the process.  Host code never passes this name to a
// kernel (on the host it is a stand-in, not a device address); it uses the
// per-device address from hipGetSymbolAddress below.
static __device__ __align__(256) float scratch[MPM_MLP_SCRATCH_FLOATS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// (with that device current) and kept.
int scratch_address(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        mpm::set_global_error("mpm_mlp_backward_noalloc: no usable current device");
        return MPM_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            mpm::set_global_error("mpm_mlp_backward_noalloc: hipGetSymbolAddress of the scratch array failed");
            return MPM_EHIP;
        }
        g_scratch_ptr[dev] = (float*)p;
    }
    *out = g_scratch_ptr[dev];
    return MPM_OK;
}

constexpr int kMaxW = 128;
constexpr int kRowsPerWave = 16;
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

struct MlpDesc {
    int L;
    int w[MPM_MLP_MAX_LAYERS + 1];    // true widths
    int wp[MPM_MLP_MAX_LAYERS + 1];   // widths padded to 16
    int offW[MPM_MLP_MAX_LAYERS], offb[MPM_MLP_MAX_LAYERS];
    long long offC[MPM_MLP_MAX_LAYERS];   // per-layer offset in the cache (per sample count n)
    int out_act;
    int hidden_act;                   // MPM_HIDDEN_TANH or MPM_HIDDEN_RELU
    float scale, shift;
    float in_scale[MPM_MLP_MAX_IN], in_shift[MPM_MLP_MAX_IN];
};

// binary32 -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ short to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One 16 x 16 tile: C[r][c] = sum_k A(r, k) * B(k, c), k < K (a multiple of
// 16).  fa(r, k) and fb(k, c) return zero outside the operands.  Lane l
// holds C[4*(l/16) + i][l%16], i = 0..3.  BF16: lane l supplies A(l%16, k)
// and B(k, l%16) for the eight k = k0 + 8*(l/16) + i of each 32-deep step
// (the same k for both operands, so the pairing is exact whatever order the
// unit sums in).
template <int BF16, class FA, class FB>
__device__ __forceinline__ f4 mfma_tile(int K, FA fa, FB fb)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    f4 c = {0.f, 0.f, 0.f, 0.f};
    if constexpr (BF16) {
        for (int k0 = 0; k0 < K; k0 += 32) {
            b8 a, b;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                a[i] = __builtin_bit_cast(__bf16, to_bf16(fa(r, k0 + 8 * q + i)));
                b[i] = __builtin_bit_cast(__bf16, to_bf16(fb(k0 + 8 * q + i, r)));
            }
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
        }
    } else {
        for (int k0 = 0; k0 < K; k0 += 4) c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa(r, k0 + q), fb(k0 + q, r), c, 0, 0, 0);
    }
    return c;
}

__device__ __forceinline__ float act_hidden(int kind, float z) { return kind == MPM_HIDDEN_RELU ? fmaxf(z, 0.f) : tanhf(z); }
// derivative of the hidden activation from its output h
__device__ __forceinline__ float dact_hidden(int kind, float h) { return kind == MPM_HIDDEN_RELU ? (h > 0.f ? 1.f : 0.f) : 1.f - h * h; }
__device__ __forceinline__ float act_out(int kind, float z) { return kind == MPM_ACT_SIGMOID ? 1.f / (1.f + expf(-z)) : z; }

constexpr int kWaves = 2;   // waves per workgroup in the row kernels

template <int BF16>
__global__ __launch_bounds__(64 * kWaves) void k_mlp_fwd(MlpDesc d, const float* __restrict__ P, long long n,
                                                 const float* __restrict__ x, float* __restrict__ y,
                                                 float* __restrict__ cache)
{
    __shared__ float sh[kWaves][2][kRowsPerWave][kMaxW + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float(*buf)[kRowsPerWave][kMaxW + 1] = sh[w];
    const long long nblk = (n + kRowsPerWave - 1) / kRowsPerWave;
    for (long long rb = (long long)blockIdx.x * kWaves + w; rb < nblk; rb += (long long)gridDim.x * kWaves) {
        const long long r0 = rb * kRowsPerWave;
        for (int i = lane; i < kRowsPerWave * d.wp[0]; i += 64) {
            int r = i / d.wp[0], k = i % d.wp[0];
            float v = 0.f;
            if (r0 + r < n && k < d.w[0]) v = d.in_scale[k] * x[k * n + r0 + r] + d.in_shift[k];
            buf[0][r][k] = v;
        }
        wave_sync();
        int cur = 0;
        for (int l = 0; l < d.L; ++l) {
            const float* W = P + d.offW[l];
            const float* bias = P + d.offb[l];
            const int win = d.w[l], wout = d.w[l + 1];
            for (int jt = 0; jt < d.wp[l + 1]; jt += 16) {
                float(*A)[kMaxW + 1] = buf[cur];
                f4 c = mfma_tile<BF16>(
                    d.wp[l], [&](int r, int k) { return k < win ? A[r][k] : 0.f; },
                    [&](int k, int col) { return (k < win && jt + col < wout) ? W[(jt + col) * win + k] : 0.f; });
                const int col = jt + (lane & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int r = 4 * (lane >> 4) + i;
                    float h = 0.f;
                    if (col < wout) {
                        float z = c[i] + bias[col];
                        h = (l < d.L - 1) ? act_hidden(d.hidden_act, z) : act_out(d.out_act, z);
                        if (r0 + r < n) cache[d.offC[l] * n + (r0 + r) * wout + col] = h;
                    }
                    buf[1 - cur][r][col] = h;
                }
            }
            wave_sync();
            cur = 1 - cur;
        }
        const int wl = d.w[d.L];
        for (int i = lane; i < kRowsPerWave * wl; i += 64) {
            int r = i / wl, c = i % wl;
            if (r0 + r < n) y[c * n + r0 + r] = d.shift + d.scale * buf[cur][r][c];
        }
        wave_sync();
    }
}

// dZ of every layer from dy, written to `work` in the cache layout.
template <int BF16>
__global__ __launch_bounds__(64 * kWaves) void k_mlp_bwd_data(MlpDesc d, const float* __restrict__ P, long long n,
                                                      const float* __restrict__ cache, const float* __restrict__ dy,
                                                      float* __restrict__ work)
{
    __shared__ float sh[kWaves][2][kRowsPerWave][kMaxW + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float(*buf)[kRowsPerWave][kMaxW + 1] = sh[w];
    const long long nblk = (n + kRowsPerWave - 1) / kRowsPerWave;
    const int L = d.L;
    for (long long rb = (long long)blockIdx.x * kWaves + w; rb < nblk; rb += (long long)gridDim.x * kWaves) {
        const long long r0 = rb * kRowsPerWave;
        const int wl = d.w[L];
        for (int i = lane; i < kRowsPerWave * d.wp[L]; i += 64) {
            int r = i / d.wp[L], c = i % d.wp[L];
            float v = 0.f;
            if (r0 + r < n && c < wl) {
                float h = cache[d.offC[L - 1] * n + (r0 + r) * wl + c];
                float g = dy[c * n + r0 + r] * d.scale;
                v = d.out_act == MPM_ACT_SIGMOID ? g * h * (1.f - h) : g;
                work[d.offC[L - 1] * n + (r0 + r) * wl + c] = v;
            }
            buf[0][r][c] = v;
        }
        wave_sync();
        int cur = 0;
        for (int l = L - 1; l >= 1; --l) {
            // dh = dz_l W_l (16 x w[l]); dz_{l-1} = dh * act'(z), from h = layer l-1 output
            const float* W = P + d.offW[l];
            const int win = d.w[l], wout = d.w[l + 1];
            for (int kt = 0; kt < d.wp[l]; kt += 16) {
                float(*A)[kMaxW + 1] = buf[cur];
                f4 c = mfma_tile<BF16>(
                    d.wp[l + 1], [&](int r, int j) { return j < wout ? A[r][j] : 0.f; },
                    [&](int j, int col) { return (j < wout && kt + col < win) ? W[j * win + kt + col] : 0.f; });
                const int col = kt + (lane & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int r = 4 * (lane >> 4) + i;
                    float v = 0.f;
                    if (col < win && r0 + r < n) {
                        float h = cache[d.offC[l - 1] * n + (r0 + r) * win + col];
                        v = c[i] * dact_hidden(d.hidden_act, h);
                        work[d.offC[l - 1] * n + (r0 + r) * win + col] = v;
                    }
                    buf[1 - cur][r][col] = v;
                }
            }
            wave_sync();
            cur = 1 - cur;
        }
        wave_sync();
    }
}

// dW_l = dZ_l^T H_l and db_l = sum dZ_l over a chunk of rows; partial
// results added to dP with atomics.  blockIdx.y = layer.
template <int BF16>
__global__ __launch_bounds__(256) void k_mlp_bwd_weights(MlpDesc d, long long n, long long chunk,
                                                         const float* __restrict__ x,
                                                         const float* __restrict__ cache,
                                                         const float* __restrict__ work, float* __restrict__ dP)
{
    const int l = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int win = d.w[l], wout = d.w[l + 1];
    const long long rbeg = (long long)blockIdx.x * chunk;
    if (rbeg >= n) return;
    const long long rend = min(rbeg + chunk, n);
    const int K = (int)(rend - rbeg);
    const int Kp = (K + 15) & ~15;
    const float* dz = work + d.offC[l] * n;
    auto hin = [&](long long r, int i) -> float {
        if (l == 0) return d.in_scale[i] * x[i * n + r] + d.in_shift[i];
        return cache[d.offC[l - 1] * n + r * win + i];
    };
    const int tiles_o = d.wp[l + 1] / 16, tiles_i = d.wp[l] / 16;
    for (int t = w; t < tiles_o * tiles_i; t += 4) {
        const int o0 = (t / tiles_i) * 16, i0 = (t % tiles_i) * 16;
        f4 c = mfma_tile<BF16>(
            Kp,
            [&](int o, int k) { return (k < K && o0 + o < wout) ? dz[(rbeg + k) * wout + o0 + o] : 0.f; },
            [&](int k, int i) { return (k < K && i0 + i < win) ? hin(rbeg + k, i0 + i) : 0.f; });
        const int ii = i0 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int oo = o0 + 4 * (lane >> 4) + q;
            if (oo < wout && ii < win) atomicAdd(&dP[d.offW[l] + oo * win + ii], c[q]);
        }
    }
    // bias: column sums of dZ over the chunk
    for (int o = threadIdx.x; o < wout; o += 256) {
        float s = 0.f;
        for (long long r = rbeg; r < rend; ++r) s += dz[r * wout + o];
        atomicAdd(&dP[d.offb[l] + o], s);
    }
}

__global__ void k_fill_f(float* p, long long n, float v)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    long long stride = (long long)gridDim.x * 256;
    for (; i < n; i += stride) p[i] = v;
}

// om1 = 1 - beta1 and om2 = 1 - beta2 are formed in binary64 by the host:
// 1 - 0.999f in binary32 would carry a 1e-5 relative error.
__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float om1, float om2, float eps, float c1,
                       float c2)
{
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + om1 * gi;
    float vi = b2 * v[i] + om2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Piecewise-constant field on an nx x ny cell grid over [lo, hi) of the first
// two coordinates; points outside take the nearest cell.
struct CellGrid {
    int nc, nx, ny;
    float lo0, lo1, inv0, inv1;
};

__device__ __forceinline__ int cell_of(const CellGrid& g, float x0, float x1)
{
    int i = (int)floorf((x0 - g.lo0) * g.inv0);
    int j = (int)floorf((x1 - g.lo1) * g.inv1);
    i = i < 0 ? 0 : (i >= g.nx ? g.nx - 1 : i);
    j = j < 0 ? 0 : (j >= g.ny ? g.ny - 1 : j);
    return j * g.nx + i;
}

__global__ void k_cell_gather(CellGrid g, long long n, const float* __restrict__ x, const float* __restrict__ table,
                              float* __restrict__ out)
{
    long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int c = cell_of(g, x[p], x[n + p]);
    for (int k = 0; k < g.nc; ++k) out[k * n + p] = table[k * g.nx * g.ny + c];
}

__global__ void k_cell_scatter(CellGrid g, long long n, const float* __restrict__ x, const float* __restrict__ dout,
                               float* __restrict__ dtable)
{
    long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    int c = cell_of(g, x[p], x[n + p]);
    for (int k = 0; k < g.nc; ++k) atomicAdd(&dtable[k * g.nx * g.ny + c], dout[k * n + p]);
}

int make_cellgrid(int nc, int nx, int ny, const double* lo, const double* hi, CellGrid* g)
{
    if (nc < 1 || nx < 1 || ny < 1 || !lo || !hi || !(hi[0] > lo[0]) || !(hi[1] > lo[1])) return MPM_EINVAL;
    g->nc = nc;
    g->nx = nx;
    g->ny = ny;
    g->lo0 = (float)lo[0];
    g->lo1 = (float)lo[1];
    g->inv0 = (float)(nx / (hi[0] - lo[0]));
    g->inv1 = (float)(ny / (hi[1] - lo[1]));
    return MPM_OK;
}

int make_desc(const mpm_mlp* net, MlpDesc* d)
{
    if (!net || net->n_layers < 1 || net->n_layers > MPM_MLP_MAX_LAYERS) return MPM_EINVAL;
    if (net->math != MPM_MLP_BF16 && net->math != MPM_MLP_F32) return MPM_EINVAL;
    if (net->out_act != MPM_ACT_NONE && net->out_act != MPM_ACT_SIGMOID) return MPM_EINVAL;
    if (net->hidden_act != MPM_HIDDEN_TANH && net->hidden_act != MPM_HIDDEN_RELU) return MPM_EINVAL;
    if (net->width[0] < 1 || net->width[0] > MPM_MLP_MAX_IN) return MPM_EINVAL;
    d->L = net->n_layers;
    int off = 0;
    long long coff = 0;
    for (int l = 0; l <= d->L; ++l) {
        int wv = net->width[l];
        if (wv < 1 || wv > kMaxW) return MPM_EINVAL;
        d->w[l] = wv;
        d->wp[l] = (wv + 15) & ~15;
    }
    for (int l = 0; l < d->L; ++l) {
        d->offW[l] = off;
        off += d->w[l + 1] * d->w[l];
        d->offb[l] = off;
        off += d->w[l + 1];
        d->offC[l] = coff;
        coff += d->w[l + 1];
    }
    d->out_act = net->out_act;
    d->hidden_act = net->hidden_act;
    d->scale = net->out_scale;
    d->shift = net->out_shift;
    for (int k = 0; k < MPM_MLP_MAX_IN; ++k) {
        d->in_scale[k] = k < d->w[0] ? net->in_scale[k] : 0.f;
        d->in_shift[k] = k < d->w[0] ? net->in_shift[k] : 0.f;
    }
    return MPM_OK;
}

unsigned grid_for(long long n)
{
    long long blk = (n + kRowsPerWave * kWaves - 1) / (kRowsPerWave * kWaves);
    return (unsigned)(blk < 4096 ? (blk > 0 ? blk : 1) : 4096);
}

}  // namespace

extern "C" {

int64_t mpm_mlp_num_params(const mpm_mlp* net)
{
    MlpDesc d;
    if (make_desc(net, &d) != MPM_OK) return -1;
    int64_t s = 0;
    for (int l = 0; l < d.L; ++l) s += (int64_t)d.w[l + 1] * (d.w[l] + 1);
    return s;
}

int64_t mpm_mlp_cache_floats(const mpm_mlp* net, int64_t n)
{
    MlpDesc d;
    if (make_desc(net, &d) != MPM_OK || n < 0) return -1;
    int64_t s = 0;
    for (int l = 1; l <= d.L; ++l) s += d.w[l];
    return s * n;
}

int mpm_mlp_forward(const mpm_mlp* net, void* hip_stream, const float* params, int64_t n, const float* x,
                    float* y, float* cache)
{
    MlpDesc d;
    int rc = make_desc(net, &d);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!params || !x || !y || !cache))) return MPM_EINVAL;
    if (n == 0) return MPM_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    if (net->math == MPM_MLP_BF16) k_mlp_fwd<1><<<grid_for(n), 64 * kWaves, 0, st>>>(d, params, n, x, y, cache);
    else k_mlp_fwd<0><<<grid_for(n), 64 * kWaves, 0, st>>>(d, params, n, x, y, cache);
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

int mpm_mlp_backward(const mpm_mlp* net, void* hip_stream, const float* params, int64_t n, const float* x,
                     const float* cache, const float* dy, float* work, float* dparams)
{
    MlpDesc d;
    int rc = make_desc(net, &d);
    if (rc) return rc;
    if (n < 0 || !dparams || (n > 0 && (!params || !x || !cache || !dy || !work))) return MPM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    long long np = mpm_mlp_num_params(net);
    k_fill_f<<<(unsigned)((np + 255) / 256 < 1024 ? (np + 255) / 256 : 1024), 256, 0, st>>>(dparams, np, 0.f);
    if (n > 0) {
        const long long chunk = 512;
        dim3 gw((unsigned)((n + chunk - 1) / chunk), (unsigned)d.L);
        if (net->math == MPM_MLP_BF16) {
            k_mlp_bwd_data<1><<<grid_for(n), 64 * kWaves, 0, st>>>(d, params, n, cache, dy, work);
            k_mlp_bwd_weights<1><<<gw, 256, 0, st>>>(d, n, chunk, x, cache, work, dparams);
        } else {
            k_mlp_bwd_data<0><<<grid_for(n), 64 * kWaves, 0, st>>>(d, params, n, cache, dy, work);
            k_mlp_bwd_weights<0><<<gw, 256, 0, st>>>(d, n, chunk, x, cache, work, dparams);
        }
    }
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

int mpm_mlp_backward_noalloc(const mpm_mlp* net, void* hip_stream, const float* params, int64_t n,
                             const float* x, const float* cache, const float* dy, float* dparams)
{
    int64_t need = mpm_mlp_cache_floats(net, n);
    if (need < 0) {
        mpm::set_global_error("mpm_mlp_backward_noalloc: invalid network description or n");
        return MPM_EINVAL;
    }
    if (need > (int64_t)MPM_MLP_SCRATCH_FLOATS) {
        mpm::set_global_error("mpm_mlp_backward_noalloc: n too large for the static scratch "
                              "(mpm_mlp_cache_floats(net, n) > MPM_MLP_SCRATCH_FLOATS)");
        return MPM_EINVAL;
    }
    float* work = nullptr;
    if (n > 0) {
        int rc = scratch_address(&work);
        if (rc) return rc;
    }
    return mpm_mlp_backward(net, hip_stream, params, n, x, cache, dy, work, dparams);
}

int mpm_cell_field_gather(void* hip_stream, int32_t nc, int32_t nx, int32_t ny, const double* host_lo,
                          const double* host_hi, int64_t n, const float* x, const float* table, float* out)
{
    CellGrid g;
    if (make_cellgrid(nc, nx, ny, host_lo, host_hi, &g) || n < 0 || (n > 0 && (!x || !table || !out)))
        return MPM_EINVAL;
    if (n == 0) return MPM_OK;
    k_cell_gather<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>(g, n, x, table, out);
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

int mpm_cell_field_scatter(void* hip_stream, int32_t nc, int32_t nx, int32_t ny, const double* host_lo,
                           const double* host_hi, int64_t n, const float* x, const float* dout, float* dtable)
{
    CellGrid g;
    if (make_cellgrid(nc, nx, ny, host_lo, host_hi, &g) || n < 0 || !dtable || (n > 0 && (!x || !dout)))
        return MPM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    long long nt = (long long)nc * nx * ny;
    k_fill_f<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(dtable, nt, 0.f);
    if (n > 0) k_cell_scatter<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(g, n, x, dout, dtable);
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

int mpm_adam_step(void* hip_stream, int64_t n, float* params, const float* grad, float* m, float* v, int32_t step,
                  double lr, double beta1, double beta2, double eps)
{
    if (n < 0 || step < 1 || (n > 0 && (!params || !grad || !m || !v))) return MPM_EINVAL;
    if (n == 0) return MPM_OK;
    float c1 = (float)(1.0 - pow(beta1, step)), c2 = (float)(1.0 - pow(beta2, step));
    k_adam<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>(n, params, grad, m, v, (float)lr,
                                                                              (float)beta1, (float)beta2,
                                                                              (float)(1.0 - beta1), (float)(1.0 - beta2),
                                                                              (float)eps, c1, c2);
    return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

}  // extern "C"
