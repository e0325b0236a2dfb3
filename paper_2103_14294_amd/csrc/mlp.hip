// Learned cost surrogate: a 2-layer MLP
//     y = b2 + sum_h W2[h] * relu(b1[h] + sum_f W1[f][h] * xn[f]),
//     xn[f] = (x[f] - xmean[f]) * xinv[f]
// that predicts the log of a per-step size of a matching order (here the
// candidates the step examines; the estimator slot of the optimiser,
// Section 3.3, which the paper leaves open).  F = 128 input features,
// H = 256 hidden units.
//
// Weights are used in BF16 (round-to-nearest-even copies of FP32 master
// weights); products and sums are FP32.  Training minimises the mean squared
// error of the standardised target (t - tmean) / tstd with Adam.
//
// Kernels:
//   k_mlp_fwd   : a workgroup per 16 samples, a thread per hidden unit; the
//                 normalised sample tile sits in LDS and each thread streams
//                 its column of W1 (coalesced across the workgroup).
//   k_mlp_bwd   : at most 64 workgroups; each walks its sample tiles and
//                 accumulates a private partial gradient (thread h owns column
//                 h of dW1); k_mlp_reduce sums the partials in a fixed order,
//                 so gradients are deterministic.
//   k_mlp_adam  : one thread per parameter; refreshes the BF16 copy.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace huge {
namespace {

constexpr int F = HUGE_MLP_F;
constexpr int H = HUGE_MLP_H;
constexpr int64_t NP = HUGE_MLP_PARAMS;
constexpr int64_t OW1 = 0, OB1 = (int64_t)F * H, OW2 = OB1 + H, OB2 = OW2 + H;
constexpr int S = 16;        // samples per tile
constexpr int kBwdGrid = 64; // workgroups of the backward pass (partial gradients)

static_assert(H == 256, "one thread per hidden unit in a 256-thread workgroup");

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FP32 -> BF16, round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float wave_sum_f32(float x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ void load_tile(float (&xs)[S][F], const float *x, const int32_t *idx, int64_t s0, int64_t B,
                                          const float *xmean, const float *xinv) {
    for (int e = threadIdx.x; e < S * F; e += H) {
        const int s = e / F, f = e % F;
        const int64_t r = s0 + s;
        float v = 0.f;
        if (r < B) {
            const int64_t row = idx ? (int64_t)idx[r] : r;
            v = (x[row * F + f] - xmean[f]) * xinv[f];
        }
        xs[s][f] = v;
    }
}

__global__ __launch_bounds__(H) void k_mlp_cast(const float *w, uint16_t *wb, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f32_to_bf16(w[i]);
}

// y[r] = yscale * (network output) + yshift; z[r][h] = pre-activations (when SAVE).
template <bool SAVE>
__global__ __launch_bounds__(H) void k_mlp_fwd(const float *x, const int32_t *idx, int64_t B, const uint16_t *wb,
                                               const float *xmean, const float *xinv, float *z, float *y, float yscale,
                                               float yshift) {
    __shared__ float xs[S][F];
    __shared__ float red[S][H / 64];
    const int h = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * S;
    load_tile(xs, x, idx, s0, B, xmean, xinv);
    __syncthreads();
    float acc[S];
    const float b1 = bf16_to_f32(wb[OB1 + h]);
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = b1;
    for (int f = 0; f < F; ++f) {
        const float w = bf16_to_f32(wb[OW1 + (int64_t)f * H + h]);
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] = fmaf(xs[s][f], w, acc[s]);
    }
    const float w2 = bf16_to_f32(wb[OW2 + h]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (SAVE && s0 + s < B) z[(s0 + s) * H + h] = acc[s];
        const float a = wave_sum_f32(fmaxf(acc[s], 0.f) * w2);
        if (__lane_id() == 0) red[s][h >> 6] = a;
    }
    __syncthreads();
    if (h < S && s0 + h < B) {
        float o = bf16_to_f32(wb[OB2]);
#pragma unroll
        for (int q = 0; q < H / 64; ++q) o += red[h][q];
        y[s0 + h] = o * yscale + yshift;
    }
}

// Partial gradients of L = (1/B) sum_r (yn[r] - (t[row] - tmean) * tinv)^2 over
// this workgroup's tiles; part[blockIdx.x] = [dW1 | db1 | dW2 | db2 | sum of
// squared errors].  Every workgroup owns at least one tile (grid <= tiles);
// thread h accumulates column h of dW1 directly in its own slab entries.
__global__ __launch_bounds__(H) void k_mlp_bwd(const float *x, const int32_t *idx, const float *t, int64_t B,
                                               const uint16_t *wb, const float *xmean, const float *xinv, float tmean,
                                               float tinv, const float *z, const float *yn, float *part) {
    __shared__ float xs[S][F];
    __shared__ float gs[S];
    __shared__ float lsum[S];
    const int h = threadIdx.x;
    float *o = part + (int64_t)blockIdx.x * (NP + 1);
    float gb1 = 0.f, gW2 = 0.f, gb2 = 0.f, loss = 0.f;
    const float w2 = bf16_to_f32(wb[OW2 + h]);
    const float invB = 1.f / (float)B;
    bool first = true;
    for (int64_t tile = blockIdx.x; tile * S < B; tile += gridDim.x) {
        const int64_t s0 = tile * S;
        load_tile(xs, x, idx, s0, B, xmean, xinv);
        if (h < S) {
            const int64_t r = s0 + h;
            float g = 0.f;
            if (r < B) {
                const int64_t row = idx ? (int64_t)idx[r] : r;
                const float d = yn[r] - (t[row] - tmean) * tinv;
                g = 2.f * d * invB;
                loss = fmaf(d, d, loss);
            }
            gs[h] = g;
        }
        __syncthreads();
        float dz[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const float zz = (s0 + s < B) ? z[(s0 + s) * H + h] : 0.f;
            gW2 = fmaf(gs[s], fmaxf(zz, 0.f), gW2);
            dz[s] = zz > 0.f ? gs[s] * w2 : 0.f;
            gb1 += dz[s];
        }
#pragma unroll 2
        for (int f = 0; f < F; ++f) {
            float a = 0.f;
#pragma unroll
            for (int s = 0; s < S; ++s) a = fmaf(xs[s][f], dz[s], a);
            float *dst = o + OW1 + (int64_t)f * H + h;
            *dst = first ? a : *dst + a;
        }
        first = false;
        if (h == 0)
            for (int s = 0; s < S; ++s) gb2 += gs[s];
        __syncthreads();
    }
    o[OB1 + h] = gb1;
    o[OW2 + h] = gW2;
    if (h < S) lsum[h] = loss;
    __syncthreads();
    if (h == 0) {
        float l = 0.f;
        for (int s = 0; s < S; ++s) l += lsum[s];
        o[OB2] = gb2;
        o[NP] = l;
    }
}

__global__ __launch_bounds__(H) void k_mlp_reduce(const float *part, int G, float *grad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NP) return;
    float s = 0.f;
    for (int b = 0; b < G; ++b) s += part[(int64_t)b * (NP + 1) + i];
    grad[i] = s;
}

// Adam (Kingma & Ba): c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ __launch_bounds__(H) void k_mlp_adam(float *w, uint16_t *wb, float *m, float *v, const float *grad,
                                                float lr, float beta1, float beta2, float eps, float c1, float c2,
                                                float *loss_acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && loss_acc) *loss_acc += grad[NP];
    if (i >= NP) return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * g;
    const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    wb[i] = f32_to_bf16(wi);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + H - 1) / H); }

// SplitMix64 step (Steele, Lea & Flood), for the epoch shuffles.
inline uint64_t sm64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Buf {
    void *p = nullptr;
    ~Buf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

huge_model *model_create() {
    huge_model *m = new huge_model();
    try {
        HUGE_HIP(hipGetDevice(&m->device));
        const uint64_t bytes = 4ull * NP * 3 + 2ull * NP + 8ull * F + 1024;
        HUGE_HIP(hipMalloc(&m->mem, bytes));
        char *c = (char *)m->mem;
        m->w = (float *)c;
        c += 4ull * NP;
        m->m = (float *)c;
        c += 4ull * NP;
        m->v = (float *)c;
        c += 4ull * NP;
        m->xmean = (float *)c;
        c += 4ull * F;
        m->xinv = (float *)c;
        c += 4ull * F;
        m->wb = (uint16_t *)(((uintptr_t)c + 255) & ~(uintptr_t)255);
        HUGE_HIP(hipMemset(m->mem, 0, bytes));
        std::vector<float> ones(F, 1.f);
        HUGE_HIP(hipMemcpy(m->xinv, ones.data(), 4ull * F, hipMemcpyHostToDevice));
    } catch (...) {
        model_free(m);
        throw;
    }
    return m;
}

void model_free(huge_model *m) {
    if (!m) return;
    if (m->mem) (void)hipFree(m->mem);
    delete m;
}

void model_set(huge_model *m, const float *params, const float *xmean, const float *xinv, float tmean, float tstd) {
    if (!(tstd > 0.f) || !std::isfinite(tmean)) HUGE_FAIL(HUGE_EINVAL, "tstd must be > 0 and tmean finite");
    if (params) {
        for (int64_t i = 0; i < NP; ++i)
            if (!std::isfinite(params[i])) HUGE_FAIL(HUGE_EINVAL, "parameter %lld is not finite", (long long)i);
        HUGE_HIP(hipMemcpy(m->w, params, 4ull * NP, hipMemcpyHostToDevice));
        HUGE_HIP(hipMemset(m->m, 0, 4ull * NP));
        HUGE_HIP(hipMemset(m->v, 0, 4ull * NP));
        m->step = 0;
        hipLaunchKernelGGL(k_mlp_cast, dim3(nblk(NP)), dim3(H), 0, nullptr, m->w, m->wb, NP);
        HUGE_HIP(hipGetLastError());
    }
    if (xmean) HUGE_HIP(hipMemcpy(m->xmean, xmean, 4ull * F, hipMemcpyHostToDevice));
    if (xinv) HUGE_HIP(hipMemcpy(m->xinv, xinv, 4ull * F, hipMemcpyHostToDevice));
    m->tmean = tmean;
    m->tstd = tstd;
    HUGE_HIP(hipDeviceSynchronize());
}

void model_get(const huge_model *m, float *params, float *xmean, float *xinv, float *tmean, float *tstd) {
    HUGE_HIP(hipDeviceSynchronize());
    if (params) HUGE_HIP(hipMemcpy(params, m->w, 4ull * NP, hipMemcpyDeviceToHost));
    if (xmean) HUGE_HIP(hipMemcpy(xmean, m->xmean, 4ull * F, hipMemcpyDeviceToHost));
    if (xinv) HUGE_HIP(hipMemcpy(xinv, m->xinv, 4ull * F, hipMemcpyDeviceToHost));
    if (tmean) *tmean = m->tmean;
    if (tstd) *tstd = m->tstd;
}

void model_forward(const huge_model *m, const float *x, int64_t B, float *y, hipStream_t st) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_mlp_fwd<false>, dim3((unsigned)((B + S - 1) / S)), dim3(H), 0, st, x, (const int32_t *)nullptr,
                       B, m->wb, m->xmean, m->xinv, (float *)nullptr, y, m->tstd, m->tmean);
    HUGE_HIP(hipGetLastError());
}

// Gradient of the loss at the current BF16 weights over all B samples.
void model_grad(const huge_model *m, const float *x, const float *t, int64_t B, float *grad_host, double *loss,
                hipStream_t st) {
    if (B <= 0) HUGE_FAIL(HUGE_EINVAL, "empty batch");
    Buf buf;
    const int G = (int)std::min<int64_t>(kBwdGrid, (B + S - 1) / S);
    const uint64_t zb = (4ull * B * H + 255) & ~255ull, yb = (4ull * B + 255) & ~255ull;
    const uint64_t pb = 4ull * G * (NP + 1), gb = 4ull * (NP + 1);
    HUGE_HIP(hipMalloc(&buf.p, zb + yb + pb + gb));
    float *z = (float *)buf.p, *yn = (float *)((char *)buf.p + zb), *part = (float *)((char *)buf.p + zb + yb);
    float *grad = (float *)((char *)part + pb);
    hipLaunchKernelGGL(k_mlp_fwd<true>, dim3((unsigned)((B + S - 1) / S)), dim3(H), 0, st, x, (const int32_t *)nullptr,
                       B, m->wb, m->xmean, m->xinv, z, yn, 1.f, 0.f);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(G), dim3(H), 0, st, x, (const int32_t *)nullptr, t, B, m->wb, m->xmean,
                       m->xinv, m->tmean, 1.f / m->tstd, z, yn, part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(nblk(NP + 1)), dim3(H), 0, st, part, G, grad);
    HUGE_HIP(hipGetLastError());
    std::vector<float> g(NP + 1);
    HUGE_HIP(hipMemcpyAsync(g.data(), grad, 4ull * (NP + 1), hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    if (grad_host) memcpy(grad_host, g.data(), 4ull * NP);
    if (loss) *loss = (double)g[NP] / (double)B;
}

// Minibatch Adam over N samples for `epochs` passes (a fresh shuffle each pass).
void model_train(huge_model *m, const float *x, const float *t, int64_t N, int epochs, int64_t batch, float lr,
                 uint64_t seed, float *loss_out, hipStream_t st) {
    if (N <= 0 || epochs <= 0 || batch <= 0) HUGE_FAIL(HUGE_EINVAL, "bad training sizes");
    if (N > INT32_MAX) HUGE_FAIL(HUGE_EINVAL, "too many samples");
    batch = std::min(batch, N);
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const int G = (int)std::min<int64_t>(kBwdGrid, (batch + S - 1) / S);
    Buf buf;
    const uint64_t ib = (4ull * N + 255) & ~255ull, zb = (4ull * batch * H + 255) & ~255ull;
    const uint64_t yb = (4ull * batch + 255) & ~255ull, pb = (4ull * G * (NP + 1) + 255) & ~255ull;
    const uint64_t gb = (4ull * (NP + 1) + 255) & ~255ull, lb = 4ull * epochs;
    HUGE_HIP(hipMalloc(&buf.p, ib + zb + yb + pb + gb + lb));
    char *c = (char *)buf.p;
    int32_t *idx = (int32_t *)c;
    float *z = (float *)(c + ib), *yn = (float *)(c + ib + zb), *part = (float *)(c + ib + zb + yb);
    float *grad = (float *)(c + ib + zb + yb + pb), *lacc = (float *)(c + ib + zb + yb + pb + gb);
    HUGE_HIP(hipMemsetAsync(lacc, 0, lb, st));
    std::vector<int32_t> perm((size_t)N);
    for (int64_t i = 0; i < N; ++i) perm[(size_t)i] = (int32_t)i;
    uint64_t rs = seed;
    const float tinv = 1.f / m->tstd;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t i = N - 1; i > 0; --i) std::swap(perm[(size_t)i], perm[(size_t)(sm64(rs) % (uint64_t)(i + 1))]);
        HUGE_HIP(hipMemcpyAsync(idx, perm.data(), 4ull * N, hipMemcpyHostToDevice, st));
        for (int64_t s0 = 0; s0 < N; s0 += batch) {
            const int64_t bs = std::min(batch, N - s0);
            const int g = (int)std::min<int64_t>(G, (bs + S - 1) / S);
            hipLaunchKernelGGL(k_mlp_fwd<true>, dim3((unsigned)((bs + S - 1) / S)), dim3(H), 0, st, x, idx + s0, bs,
                               m->wb, m->xmean, m->xinv, z, yn, 1.f, 0.f);
            hipLaunchKernelGGL(k_mlp_bwd, dim3(g), dim3(H), 0, st, x, idx + s0, t, bs, m->wb, m->xmean, m->xinv,
                               m->tmean, tinv, z, yn, part);
            hipLaunchKernelGGL(k_mlp_reduce, dim3(nblk(NP + 1)), dim3(H), 0, st, part, g, grad);
            m->step += 1;
            const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)m->step)));
            const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)m->step)));
            hipLaunchKernelGGL(k_mlp_adam, dim3(nblk(NP)), dim3(H), 0, st, m->w, m->wb, m->m, m->v, grad, lr, beta1,
                               beta2, eps, c1, c2, lacc + ep);
            HUGE_HIP(hipGetLastError());
        }
        // the host permutation is rewritten next epoch: wait for its copy
        HUGE_HIP(hipStreamSynchronize(st));
    }
    std::vector<float> l((size_t)epochs);
    HUGE_HIP(hipMemcpyAsync(l.data(), lacc, lb, hipMemcpyDeviceToHost, st));
    HUGE_HIP(hipStreamSynchronize(st));
    if (loss_out)
        for (int ep = 0; ep < epochs; ++ep) loss_out[ep] = l[(size_t)ep] / (float)N;
}

}  // namespace huge
