// Training and batch inference of the learned proposal correction.
//
//  k_mlp_features  features of every site of a batch of configurations
//                  (couplings, already-sampled spins, low-chi logit)
//  k_mlp_grad      forward + backward of the soft-target cross-entropy for
//                  64 rows per workgroup; writes one partial gradient per
//                  workgroup (no float atomics: the sum order is fixed)
//  k_mlp_reduce    sums the partial gradients in workgroup order, then
//                  optionally applies one Adam step (Kingma & Ba, 2015)
//  k_mlp_forward   the correction d for a batch of feature rows
#include <mutex>

#include "mlp_device.hpp"

namespace tnmc {

constexpr int GR = 64;   // rows per gradient workgroup

__global__ void __launch_bounds__(256)
k_mlp_features(const InstDesc *__restrict__ desc, int n_samples, const uint64_t *__restrict__ spins,
               const float *__restrict__ logits, const float *__restrict__ Jh_all,
               const float *__restrict__ Jv_all, float *__restrict__ feat) {
    const int inst = blockIdx.z, n = blockIdx.y;
    const InstDesc d = desc[inst];
    const int L = d.L, W = d.W;
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= L * L) return;
    const int r = site / L, c = site % L;
    const uint64_t *s = spins + (size_t)n_samples * d.word_prefix + (size_t)n * L * W;
    const size_t row = (size_t)n_samples * d.site_prefix + (size_t)n * L * L + site;
    auto spin = [&](int rr, int cc) -> float { return ((s[(size_t)rr * W + (cc >> 6)] >> (cc & 63)) & 1) ? 1.f : -1.f; };
    float x[MLP_IN];
    mlp_features(Jh_all + d.off_h, Jv_all + d.off_v, L, r, c, spin, logits[row], x);
    float4 *out = reinterpret_cast<float4 *>(feat + row * MLP_IN);
#pragma unroll
    for (int k = 0; k < MLP_IN / 4; ++k) out[k] = make_float4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]);
}

__device__ __forceinline__ float sigm(float z) { return 0.5f * (1.f + tanhf(0.5f * z)); }

__global__ void __launch_bounds__(GR)
k_mlp_grad(const float *__restrict__ P, int n, const float *__restrict__ feat,
           const float *__restrict__ logit_lo, const float *__restrict__ target,
           float *__restrict__ partial, float *__restrict__ loss_partial) {
    extern __shared__ float sm[];
    float *Ps = sm;                          // MLP_NPARAM (+3 pad)
    float *X = Ps + MLP_NPARAM + 3;          // [GR][65]
    float *H1 = X + GR * 65;
    float *GA1 = H1 + GR * 65;
    float *GA2 = GA1 + GR * 65;
    float *GH2 = GA2 + GR * 65;              // g_d * h2
    float *GD = GH2 + GR * 65;               // [GR]
    float *LS = GD + GR;                     // [GR]
    const int t = threadIdx.x;
    for (int e = t; e < MLP_NPARAM; e += GR) Ps[e] = P[e];
    const int row = blockIdx.x * GR + t;
    const bool ok = row < n;
    float x[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = ok ? feat[(size_t)row * MLP_IN + i] : 0.f;
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) X[t * 65 + i] = x[i];
    __syncthreads();
    float h1[MLP_H], h2[MLP_H];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        float a = Ps[MLP_OFF_B1 + o];
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) a += Ps[MLP_OFF_W1 + o * MLP_IN + i] * x[i];
        h1[o] = tanhf(a);
        H1[t * 65 + o] = h1[o];
    }
    float dd = Ps[MLP_OFF_B3];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        float a = Ps[MLP_OFF_B2 + o];
#pragma unroll
        for (int i = 0; i < MLP_H; ++i) a += Ps[MLP_OFF_W2 + o * MLP_H + i] * h1[i];
        h2[o] = tanhf(a);
        dd += Ps[MLP_OFF_W3 + o] * h2[o];
    }
    float gd = 0.f, lossv = 0.f;
    if (ok) {
        const float z = logit_lo[row] + dd;
        const float tt = sigm(target[row]);
        gd = (sigm(z) - tt) / (float)n;
        lossv = (fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)))) - tt * z;
    }
    GD[t] = gd;
    LS[t] = lossv;
    float ga2[MLP_H];
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        ga2[o] = gd * Ps[MLP_OFF_W3 + o] * (1.f - h2[o] * h2[o]);
        GA2[t * 65 + o] = ga2[o];
        GH2[t * 65 + o] = gd * h2[o];
    }
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) {
        float g = 0.f;
#pragma unroll
        for (int o = 0; o < MLP_H; ++o) g += ga2[o] * Ps[MLP_OFF_W2 + o * MLP_H + i];
        GA1[t * 65 + i] = g * (1.f - h1[i] * h1[i]);
    }
    __syncthreads();
    // this workgroup's gradient, summed over its rows in row order
    float *out = partial + (size_t)blockIdx.x * MLP_NPARAM;
    for (int p = t; p < MLP_NPARAM; p += GR) {
        float g = 0.f;
        if (p < MLP_OFF_B1) {
            const int o = p / MLP_IN, i = p % MLP_IN;
            for (int rr = 0; rr < GR; ++rr) g += GA1[rr * 65 + o] * X[rr * 65 + i];
        } else if (p < MLP_OFF_W2) {
            const int o = p - MLP_OFF_B1;
            for (int rr = 0; rr < GR; ++rr) g += GA1[rr * 65 + o];
        } else if (p < MLP_OFF_B2) {
            const int o = (p - MLP_OFF_W2) / MLP_H, i = (p - MLP_OFF_W2) % MLP_H;
            for (int rr = 0; rr < GR; ++rr) g += GA2[rr * 65 + o] * H1[rr * 65 + i];
        } else if (p < MLP_OFF_W3) {
            const int o = p - MLP_OFF_B2;
            for (int rr = 0; rr < GR; ++rr) g += GA2[rr * 65 + o];
        } else if (p < MLP_OFF_B3) {
            const int i = p - MLP_OFF_W3;
            for (int rr = 0; rr < GR; ++rr) g += GH2[rr * 65 + i];
        } else {
            for (int rr = 0; rr < GR; ++rr) g += GD[rr];
        }
        out[p] = g;
    }
    if (t == 0) {
        float l = 0.f;
        for (int rr = 0; rr < GR; ++rr) l += LS[rr];
        loss_partial[blockIdx.x] = l;
    }
}

__global__ void __launch_bounds__(256)
k_mlp_reduce(const float *__restrict__ partial, const float *__restrict__ loss_partial, int nblk, int n,
             float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
             float *__restrict__ grad_out, float *__restrict__ loss_out, float lr, int step, int update) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) {
        double l = 0.0;
        for (int b = 0; b < nblk; ++b) l += loss_partial[b];
        *loss_out = (float)(l / n);
    }
    if (p >= MLP_NPARAM) return;
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += partial[(size_t)b * MLP_NPARAM + p];
    if (grad_out) grad_out[p] = g;
    if (update) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mm = b1 * m[p] + (1.f - b1) * g;
        const float vv = b2 * v[p] + (1.f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float mh = mm / (1.f - powf(b1, (float)step));
        const float vh = vv / (1.f - powf(b2, (float)step));
        P[p] -= lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ void __launch_bounds__(256)
k_mlp_forward(const float *__restrict__ P, int n, const float *__restrict__ feat, int bf16,
              float *__restrict__ d_out) {
    __shared__ float Ps[MLP_NPARAM];
    for (int e = threadIdx.x; e < MLP_NPARAM; e += blockDim.x)
        Ps[e] = bf16 ? __bfloat162float(__float2bfloat16(P[e])) : P[e];
    __syncthreads();
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    float x[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = feat[(size_t)row * MLP_IN + i];
    d_out[row] = mlp_forward(Ps, x);
}

// Scratch of the allocation-free training step: the per-workgroup partial
// gradients and losses of up to kMlpStaticRows rows, one copy per GPU for the
// life of the process.  Host code never passes this name to a kernel: it
// takes the device address from mlp_static_scratch().
constexpr int kMlpStaticRows = 16384;
constexpr size_t kMlpStaticFloats = (size_t)(kMlpStaticRows / GR) * (MLP_NPARAM + 1);
static __device__ __align__(256) float scratch[kMlpStaticFloats];

// Device address of this GPU's copy of the static scratch, looked up once per
// device (with that device current) and kept.  Returns the HIP error of the
// lookup; *out receives the address and *floats its capacity.
hipError_t mlp_static_scratch(float **out, size_t *floats) {
    static std::mutex mu;
    static float *addr[256] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 256) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<float *>(ptr);
    }
    *out = addr[dev];
    *floats = kMlpStaticFloats;
    return hipSuccess;
}

int mlp_static_max_rows() { return kMlpStaticRows; }

size_t mlp_grad_lds_bytes() { return sizeof(float) * (MLP_NPARAM + 3 + 5 * GR * 65 + 2 * GR); }

hipError_t launch_mlp_features(const InstDesc *desc, int B, int Lmax, int n_samples, const uint64_t *spins,
                               const float *logits, const float *Jh, const float *Jv, float *feat, hipStream_t st) {
    dim3 grid((Lmax * Lmax + 255) / 256, n_samples, B);
    hipLaunchKernelGGL(k_mlp_features, grid, dim3(256), 0, st, desc, n_samples, spins, logits, Jh, Jv, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, int n, const float *feat, const float *lo, const float *tgt,
                           float *partial, float *loss_partial, float *m, float *v, float *grad_out,
                           float *loss_out, float lr, int step, int update, float *Pw, hipStream_t st) {
    const int nblk = (n + GR - 1) / GR;
    const size_t lds = mlp_grad_lds_bytes();
    hipError_t e = hipFuncSetAttribute((const void *)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(GR), lds, st, P, n, feat, lo, tgt, partial, loss_partial);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, partial, loss_partial,
                       nblk, n, Pw, m, v, grad_out, loss_out, lr, step, update);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *P, int n, const float *feat, int bf16, float *d, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, st, P, n, feat, bf16, d);
    return hipGetLastError();
}

}  // namespace tnmc
