// Learned warm start: a per-factor-column 1-D CNN (four circular width-5 convolutions,
// channels 3 -> 32 -> 32 -> 32 -> 1, ReLU after the first three) whose output predicts the
// next step's factor column; ALS then refines that guess (Section 3.1 starts the
// sequential minimisation of a step from a guess of f_{n+1}).
//
// Storage: activations and gradients as BF16 [sample][position][channel] (channels padded to
// a multiple of 8, so eight channels are one 16-byte LDS read); weights as BF16 matrices
// W[out][k], k = t * Cin_pad + ci; sums in FP32 on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16],
// j < 8, and holds D[4 (l / 16) + v][l % 16]).  FP32 master weights with Adam moments.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <math.h>
#include "warmstart_internal.h"

namespace cpws {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int TPB = 256;   // threads per workgroup (4 waves)

__device__ __forceinline__ u16 f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                          // round to nearest even
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float f2bf_round_float(float x) { return bf2f(f2bf(x)); }

__device__ __forceinline__ bf8 ld8(const u16* p) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    bf8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

__device__ __forceinline__ int wrapn(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// ---------------------------------------------------------------------------------------
// Circular convolution as an implicit GEMM, one sample per workgroup:
//   out[i][o] = sum_{t < 5, c < CiP} W[o][t CiP + c] in[(i + dir (t - 2)) mod n][c]
// dir = +1: forward layer (o = output channel); dir = -1: the adjoint in the input (the
// backward data pass, o = input channel of the layer, W holding the transposed taps).
// Epilogue by mode: CONV_RELU: + bias, ReLU, BF16 [n][NoP]; CONV_LINEAR: + bias, FP32 y[n]
// (output channel 0); CONV_MASK: times [mask[i][o] > 0], BF16 [n][NoP].
// ---------------------------------------------------------------------------------------
enum { CONV_RELU = 0, CONV_LINEAR = 1, CONV_MASK = 2 };

template <int NT>   // 16-column output tiles (NoP = 16 NT)
__global__ void __launch_bounds__(TPB) conv_mfma(const u16* __restrict__ in, int CiP, int n, int dir,
                                                 const u16* __restrict__ W, int Kp, const float* __restrict__ bias,
                                                 int No, int mode, const u16* __restrict__ mask, int maskP,
                                                 u16* __restrict__ out, int outP, float* __restrict__ yout) {
    extern __shared__ __attribute__((aligned(16))) unsigned char ws_smem[];
    u16* Xs = reinterpret_cast<u16*>(ws_smem);             // [n][CiP]
    u16* Ws = Xs + n * CiP;                                 // [16 NT][Kp]
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const u16* src = in + (int64_t)b * n * CiP;
    {
        const int nv = n * CiP / 8;                         // 16-byte vectors
        const uint4* s4 = reinterpret_cast<const uint4*>(src);
        uint4* d4 = reinterpret_cast<uint4*>(Xs);
        for (int t = tid; t < nv; t += TPB) d4[t] = s4[t];
        const int nw = 16 * NT * Kp / 8;
        const uint4* w4 = reinterpret_cast<const uint4*>(W);
        uint4* x4 = reinterpret_cast<uint4*>(Ws);
        for (int t = tid; t < nw; t += TPB) x4[t] = w4[t];
    }
    __syncthreads();
    const int g = lane >> 4, cc = lane & 15;
    const int nstrip = n >> 4;
    const int ksteps = Kp >> 5;
    for (int strip = wave; strip < nstrip; strip += TPB / 64) {
        f4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        const int i = strip * 16 + cc;
        for (int s = 0; s < ksteps; ++s) {
            const int k0 = 32 * s + 8 * g;
            const int tap = k0 / CiP, c0 = k0 - tap * CiP;
            bf8 a;
            if (tap < 5) {
                a = ld8(Xs + wrapn(i + dir * (tap - 2), n) * CiP + c0);
            } else {
                const uint4 z = {0u, 0u, 0u, 0u};
                __builtin_memcpy(&a, &z, 16);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf8 bw = ld8(Ws + (t * 16 + cc) * Kp + k0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int o = t * 16 + cc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = strip * 16 + 4 * g + v;
                float val = acc[t][v];
                if (mode == CONV_RELU) {
                    if (o < outP) {
                        val = (o < No) ? fmaxf(val + bias[o], 0.f) : 0.f;
                        out[((int64_t)b * n + row) * outP + o] = f2bf(val);
                    }
                } else if (mode == CONV_LINEAR) {
                    if (o == 0) yout[(int64_t)b * n + row] = val + bias[0];
                } else {
                    if (o < outP) {
                        const float m = (o < No) ? bf2f(mask[((int64_t)b * n + row) * maskP + o]) : 0.f;
                        out[((int64_t)b * n + row) * outP + o] = f2bf(m > 0.f ? val : 0.f);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Weight gradient of one layer over a group of samples per workgroup:
//   dW[o][t CiP + c] = sum_{b, i} g[b][i][o] x[b][(i + t - 2) mod n][c],   db[o] = sum g[b][i][o]
// as D[o][k] with the positions as the contraction: A[o][i] from G transposed in LDS,
// B[i][k] from five tap-shifted, channel-major copies of x in LDS (16-byte aligned reads).
// Each workgroup writes FP32 partials part[wg][MP][Kp] and dbp[wg][MP].
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) wgrad_mfma(const u16* __restrict__ gin, int GoP, int No, const u16* __restrict__ x,
                                                  int CiP, int n, int B, int per_wg, int MP, int Kp,
                                                  float* __restrict__ part, float* __restrict__ dbp) {
    extern __shared__ __attribute__((aligned(16))) unsigned char ws_smem[];
    u16* Gt = reinterpret_cast<u16*>(ws_smem);        // [MP][n]
    u16* Xt = Gt + MP * n;                            // [5][CiP][n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, cc = lane & 15;
    const int TMt = MP / 16, TNt = Kp / 16;
    const int ntile = TMt * TNt;
    constexpr int TPW = 8;   // tiles per wave (MP <= 32, Kp <= 256 -> at most 32 tiles)
    f4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;
    const int b0 = blockIdx.x * per_wg, b1 = min(B, b0 + per_wg);
    for (int b = b0; b < b1; ++b) {
        __syncthreads();
        for (int t = tid; t < MP * n; t += TPB) {
            const int o = t / n, i = t - o * n;
            Gt[t] = (o < No && o < GoP) ? gin[((int64_t)b * n + i) * GoP + o] : (u16)0;
        }
        for (int t = tid; t < 5 * CiP * n; t += TPB) {
            const int tap = t / (CiP * n), rem = t - tap * CiP * n;
            const int c = rem / n, i = rem - c * n;
            Xt[t] = x[((int64_t)b * n + wrapn(i + tap - 2, n)) * CiP + c];
        }
        __syncthreads();
        // bias gradient: thread o sums its channel
        if (tid < MP) {
            float s = 0.f;
            for (int i = 0; i < n; ++i) s += bf2f(Gt[tid * n + i]);
            dbacc += s;
        }
        for (int i0 = 0; i0 < n; i0 += 32) {
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int tile = wave + (TPB / 64) * u;
                if (tile < ntile) {
                    const int tm = tile % TMt, tn = tile / TMt;
                    const int kcol = tn * 16 + cc;           // this lane's column k of B
                    const int tap = kcol / CiP, c = kcol - tap * CiP;
                    const bf8 a = ld8(Gt + (tm * 16 + cc) * n + i0 + 8 * g);
                    bf8 bv;
                    if (tap < 5) {
                        bv = ld8(Xt + (tap * CiP + c) * n + i0 + 8 * g);
                    } else {
                        const uint4 z = {0u, 0u, 0u, 0u};
                        __builtin_memcpy(&bv, &z, 16);
                    }
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[u], 0, 0, 0);
                }
            }
        }
    }
    float* pp = part + (int64_t)blockIdx.x * MP * Kp;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int tile = wave + (TPB / 64) * u;
        if (tile < ntile) {
            const int tm = tile % TMt, tn = tile / TMt;
#pragma unroll
            for (int v = 0; v < 4; ++v) pp[(tm * 16 + 4 * g + v) * Kp + tn * 16 + cc] = acc[u][v];
        }
    }
    if (tid < MP) dbp[(int64_t)blockIdx.x * MP + tid] = dbacc;
}

// Sum of the workgroup partials (fixed order) into the natural FP32 gradient layout
// dW[o][c][t] (o < No, c < Ci) followed by db[o].
__global__ void wgrad_reduce(const float* __restrict__ part, const float* __restrict__ dbp, int nwg, int MP, int Kp,
                             int No, int Ci, int CiP, float* __restrict__ grad) {
    const int nw = No * Ci * 5;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nw) {
        const int o = t / (Ci * 5), rem = t - o * Ci * 5;
        const int c = rem / 5, tap = rem - c * 5;
        const int k = tap * CiP + c;
        float s = 0.f;
        for (int w = 0; w < nwg; ++w) s += part[((int64_t)w * MP + o) * Kp + k];
        grad[t] = s;
    } else if (t < nw + No) {
        const int o = t - nw;
        float s = 0.f;
        for (int w = 0; w < nwg; ++w) s += dbp[(int64_t)w * MP + o];
        grad[t] = s;
    }
}

// ---------------------------------------------------------------------------------------
// inputs, targets, loss, output
// ---------------------------------------------------------------------------------------
// x FP32 [B][3][n] (the natural layout) -> BF16 [B][n][8]
__global__ void pack_input(const float* __restrict__ x, int B, int n, u16* __restrict__ act0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * n * 8) return;
    const int c = (int)(t & 7);
    const int64_t bi = t >> 3;
    const int b = (int)(bi / n), i = (int)(bi - (int64_t)b * n);
    act0[t] = (c < 3) ? f2bf(x[((int64_t)b * 3 + c) * n + i]) : (u16)0;
}

// Output scale of the network's correction (a power of two: exact in BF16, FP32 and FP64).
// The correction of the linear extrapolation is a small fraction of the column; the scale
// lets the network produce it as outputs of order one.
constexpr double OUT_SCALE = 1.0 / 4096.0;

// Samples from columns of factor panels: sample s = (u_prev, u_cur[, u_next]) rows of n
// values.  One workgroup per sample: the RMS scale, the BF16 input channels and (training)
// the FP32 target (u_next - 2 u_cur + u_prev) / (OUT_SCALE s), the second difference in
// time that corrects the linear extrapolation.  Column sources come through a table of
// pointers.
__global__ void __launch_bounds__(TPB) make_samples(const double* const* __restrict__ prev, const double* const* __restrict__ cur,
                                                    const double* const* __restrict__ next, const double* __restrict__ coef,
                                                    int n, u16* __restrict__ act0, float* __restrict__ target,
                                                    double* __restrict__ scale) {
    __shared__ double red[TPB / 64];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double* up = prev[b];
    const double* uc = cur[b];
    double s2 = 0.0;
    for (int i = tid; i < n; i += TPB) s2 += uc[i] * uc[i];
    for (int off = 32; off > 0; off >>= 1) s2 += __shfl_down(s2, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = s2;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < TPB / 64; ++w) tot += red[w];
    double s = sqrt(tot / n);
    if (!(s > 0.0)) s = 1.0;
    const double inv = 1.0 / s;
    const float cf = (float)coef[b];
    for (int i = tid; i < n; i += TPB) {
        u16* a = act0 + ((int64_t)b * n + i) * 8;
        a[0] = f2bf((float)(up[i] * inv));
        a[1] = f2bf((float)(uc[i] * inv));
        a[2] = f2bf(cf);
#pragma unroll
        for (int c = 3; c < 8; ++c) a[c] = 0;
        if (target) target[(int64_t)b * n + i] = (float)((next[b][i] - (2.0 * uc[i] - up[i])) * (inv / OUT_SCALE));
    }
    if (tid == 0 && scale) scale[b] = s;
}

// dy = 2 (y - target) / (B n) as BF16 channel 0 of [B][n][8]; per-block partial sums of the
// squared error (reduced on the host side of the library in fixed order).
__global__ void __launch_bounds__(TPB) mse_grad(const float* __restrict__ y, const float* __restrict__ target, int64_t total,
                                                u16* __restrict__ g4, float* __restrict__ lpart) {
    __shared__ float red[TPB / 64];
    const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
    float e2 = 0.f;
    if (t < total) {
        const float d = y[t] - target[t];
        e2 = d * d;
        u16* gp = g4 + t * 8;
        gp[0] = f2bf(2.f * d / (float)total);
#pragma unroll
        for (int c = 1; c < 8; ++c) gp[c] = 0;
    }
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_down(e2, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < TPB / 64; ++w) s += red[w];
        lpart[blockIdx.x] = s;
    }
}

// Next columns 2 u_cur - u_prev + OUT_SCALE s y (the linear extrapolation and the
// network's correction) into the output panels (pointer tables per sample; dst may be
// u_cur).
__global__ void finish_guess(const double* const* __restrict__ prev, const double* const* __restrict__ cur,
                             double* const* __restrict__ dst, const double* __restrict__ scale,
                             const float* __restrict__ y, int n, int B) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * n) return;
    const int b = (int)(t / n), i = (int)(t - (int64_t)b * n);
    dst[b][i] = (2.0 * cur[b][i] - prev[b][i]) + (OUT_SCALE * scale[b]) * (double)y[t];
}

// Adam on the FP32 master parameters (natural order), then the BF16 matrices of every
// layer: forward Wf[o][t CiP + c] and adjoint Wb[c][t CoP + o].
__global__ void adam_update(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int np, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

__global__ void pack_weights(const float* __restrict__ p, LayerDesc L, u16* __restrict__ wf, u16* __restrict__ wb,
                             float* __restrict__ bias) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const float* W = p + L.off;
    // forward matrix [16 NTf][Kpf]
    const int nf = L.NoPf * L.Kpf;
    if (t < nf) {
        const int o = t / L.Kpf, k = t - o * L.Kpf;
        const int tap = k / L.CiP, c = k - tap * L.CiP;
        float w = 0.f;
        if (o < L.Co && tap < 5 && c < L.Ci) w = W[(o * L.Ci + c) * 5 + tap];
        wf[t] = f2bf(w);
    }
    const int nb = L.NoPb * L.Kpb;
    if (t < nb) {
        const int c = t / L.Kpb, k = t - c * L.Kpb;
        const int tap = k / L.CoP, o = k - tap * L.CoP;
        float w = 0.f;
        if (c < L.Ci && tap < 5 && o < L.Co) w = W[(o * L.Ci + c) * 5 + tap];
        wb[t] = f2bf(w);
    }
    if (t < L.Co) bias[t] = f2bf_round_float(p[L.off + L.Co * L.Ci * 5 + t]);
}

}  // namespace cpws

// =======================================================================================
// host side: the cp_ws_* entry points of include/cpals_ws.h
// =======================================================================================
#include <vector>
#include <string>
#include <algorithm>
#include "../../include/cpals_ws.h"

namespace cpals {
hipStream_t handle_stream(cp_handle h);
cp_status handle_fail(cp_handle h, cp_status st, const char* msg);
cp_status handle_check_tensor(cp_handle h, const cp_tensor* t, const char* name);
}  // namespace cpals

using cpws::u16;

struct cp_ws_net_s {
    int n = 0, maxB = 0, t = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    u16* wf[cpws::NLAYER] = {};
    u16* wb[cpws::NLAYER] = {};
    float* bias[cpws::NLAYER] = {};
    u16* act[cpws::NLAYER] = {};   // inputs of the layers: [maxB][n][CiP]
    u16* gb[2] = {};               // gradient ping-pong [maxB][n][32]
    u16* g4 = nullptr;             // output gradient [maxB][n][8]
    float *y = nullptr, *target = nullptr, *part = nullptr, *dbp = nullptr, *lpart = nullptr;
    double* scale = nullptr;
    const double** tab = nullptr;  // [3][maxB] column pointers (prev, cur, next)
    double** dst = nullptr;        // [maxB] output column pointers
    double* coef = nullptr;        // [maxB]
    std::vector<void*> allocs;
};

namespace {

constexpr int NWG_MAX = 256;

#define WS_TRY(expr, what)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return cpals::handle_fail(h, CP_ERR_HIP, (std::string(what) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

template <class T>
hipError_t ws_alloc(cp_ws_net net, T** out, size_t count) {
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        net->allocs.push_back(ptr);
        *out = reinterpret_cast<T*>(ptr);
    }
    return e;
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }

hipError_t launch_conv(int NT, const u16* in, int CiP, int n, int dir, const u16* W, int Kp, const float* bias, int No,
                       int mode, const u16* mask, int maskP, u16* out, int outP, float* y, int B, hipStream_t st) {
    const size_t smem = ((size_t)n * CiP + (size_t)16 * NT * Kp) * sizeof(u16);
    const void* fn = NT == 1 ? (const void*)cpws::conv_mfma<1> : (const void*)cpws::conv_mfma<2>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    if (NT == 1)
        hipLaunchKernelGGL(cpws::conv_mfma<1>, dim3(B), dim3(cpws::TPB), smem, st, in, CiP, n, dir, W, Kp, bias, No, mode,
                           mask, maskP, out, outP, y);
    else
        hipLaunchKernelGGL(cpws::conv_mfma<2>, dim3(B), dim3(cpws::TPB), smem, st, in, CiP, n, dir, W, Kp, bias, No, mode,
                           mask, maskP, out, outP, y);
    return hipGetLastError();
}

hipError_t launch_wgrad(cp_ws_net net, const u16* gin, int GoP, int l, const u16* x, int B, hipStream_t st) {
    const cpws::LayerDesc L = cpws::layer_desc(l);
    const int n = net->n;
    const int MP = (L.Co + 15) / 16 * 16;
    const int per = ceil_div(B, NWG_MAX);
    const int nwg = ceil_div(B, per);
    const size_t smem = ((size_t)MP * n + (size_t)5 * L.CiP * n) * sizeof(u16);
    hipError_t e = hipFuncSetAttribute((const void*)cpws::wgrad_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cpws::wgrad_mfma, dim3(nwg), dim3(cpws::TPB), smem, st, gin, GoP, L.Co, x, L.CiP, n, B, per, MP,
                       L.Kpf, net->part, net->dbp);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nout = L.Co * L.Ci * 5 + L.Co;
    hipLaunchKernelGGL(cpws::wgrad_reduce, dim3(ceil_div(nout, 256)), dim3(256), 0, st, net->part, net->dbp, nwg, MP, L.Kpf,
                       L.Co, L.Ci, L.CiP, net->grad + L.off);
    return hipGetLastError();
}

hipError_t pack_all(cp_ws_net net, hipStream_t st) {
    for (int l = 0; l < cpws::NLAYER; ++l) {
        const cpws::LayerDesc L = cpws::layer_desc(l);
        const int nt = std::max(std::max(L.NoPf * L.Kpf, L.NoPb * L.Kpb), L.Co);
        hipLaunchKernelGGL(cpws::pack_weights, dim3(ceil_div(nt, 256)), dim3(256), 0, st, net->p, L, net->wf[l], net->wb[l],
                           net->bias[l]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// act[0] holds the inputs of B samples; all activations and y follow.
hipError_t forward_all(cp_ws_net net, int B, hipStream_t st) {
    const int n = net->n;
    for (int l = 0; l < cpws::NLAYER; ++l) {
        const cpws::LayerDesc L = cpws::layer_desc(l);
        const bool last = l == cpws::NLAYER - 1;
        hipError_t e = launch_conv(L.NoPf / 16, net->act[l], L.CiP, n, +1, net->wf[l], L.Kpf, net->bias[l], L.Co,
                                   last ? cpws::CONV_LINEAR : cpws::CONV_RELU, nullptr, 0,
                                   last ? nullptr : net->act[l + 1], last ? 0 : cpws::layer_desc(l + 1).CiP, net->y, B, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// loss gradient from net->y and target, then every layer's parameter gradient into net->grad;
// the per-block squared errors are left in net->lpart (returns their count).
hipError_t backward_all(cp_ws_net net, const float* target, int B, hipStream_t st, int* nblk) {
    const int n = net->n;
    const int64_t total = (int64_t)B * n;
    const int blocks = (int)((total + cpws::TPB - 1) / cpws::TPB);
    hipLaunchKernelGGL(cpws::mse_grad, dim3(blocks), dim3(cpws::TPB), 0, st, net->y, target, total, net->g4, net->lpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    *nblk = blocks;
    const u16* g = net->g4;
    int gP = 8;
    int pp = 0;
    for (int l = cpws::NLAYER - 1; l >= 0; --l) {
        const cpws::LayerDesc L = cpws::layer_desc(l);
        e = launch_wgrad(net, g, gP, l, net->act[l], B, st);
        if (e != hipSuccess) return e;
        if (l == 0) break;
        // gradient of the layer input, masked by the ReLU that produced it
        u16* out = net->gb[pp];
        e = launch_conv(L.NoPb / 16, g, gP, n, -1, net->wb[l], L.Kpb, nullptr, L.Ci, cpws::CONV_MASK, net->act[l], L.CiP,
                        out, L.CiP, nullptr, B, st);
        if (e != hipSuccess) return e;
        g = out;
        gP = L.CiP;
        pp ^= 1;
    }
    return hipSuccess;
}

cp_status read_loss(cp_handle h, cp_ws_net net, int nblk, int64_t total, float* loss_host) {
    std::vector<float> lp(nblk);
    WS_TRY(hipMemcpyAsync(lp.data(), net->lpart, nblk * sizeof(float), hipMemcpyDeviceToHost, cpals::handle_stream(h)),
           "hipMemcpyAsync(loss)");
    WS_TRY(hipStreamSynchronize(cpals::handle_stream(h)), "hipStreamSynchronize");
    double s = 0.0;
    for (float v : lp) s += v;
    if (loss_host) *loss_host = (float)(s / (double)total);
    return CP_OK;
}

cp_status check_batch(cp_handle h, cp_ws_net net, int B) {
    if (!net) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null network");
    if (B < 1) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "batch must be >= 1");
    if (B > net->maxB) return cpals::handle_fail(h, CP_ERR_SHAPE, "batch larger than the network's max_batch");
    return CP_OK;
}

}  // namespace

extern "C" {

int32_t cp_ws_num_params(void) { return cpws::N_PARAMS; }

cp_status cp_ws_create(cp_handle h, const float* params_host, int32_t n, int32_t max_batch, cp_ws_net* out) {
    if (!h || !params_host || !out) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20)) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "max_batch out of range");
    if (n < 16 || n % 16 != 0 || n > 1024)
        return cpals::handle_fail(h, CP_ERR_UNSUPPORTED, "n must be a multiple of 16 in [16, 1024]");
    cp_ws_net net = new (std::nothrow) cp_ws_net_s;
    if (!net) return cpals::handle_fail(h, CP_ERR_HIP, "host allocation");
    net->n = n;
    net->maxB = max_batch;
    const size_t nb = (size_t)max_batch * n;
    hipError_t e = hipSuccess;
    auto A = [&](auto** ptr, size_t count) {
        if (e == hipSuccess) e = ws_alloc(net, ptr, count);
    };
    A(&net->p, cpws::N_PARAMS);
    A(&net->m, cpws::N_PARAMS);
    A(&net->v, cpws::N_PARAMS);
    A(&net->grad, cpws::N_PARAMS);
    for (int l = 0; l < cpws::NLAYER; ++l) {
        const cpws::LayerDesc L = cpws::layer_desc(l);
        A(&net->wf[l], (size_t)L.NoPf * L.Kpf);
        A(&net->wb[l], (size_t)L.NoPb * L.Kpb);
        A(&net->bias[l], L.Co);
        A(&net->act[l], nb * L.CiP);
    }
    A(&net->gb[0], nb * cpws::CH_HID);
    A(&net->gb[1], nb * cpws::CH_HID);
    A(&net->g4, nb * 8);
    A(&net->y, nb);
    A(&net->target, nb);
    A(&net->scale, max_batch);
    A(&net->part, (size_t)NWG_MAX * 32 * 256);
    A(&net->dbp, (size_t)NWG_MAX * 32);
    A(&net->lpart, (nb + cpws::TPB - 1) / cpws::TPB);
    A(&net->tab, (size_t)3 * max_batch);
    A(&net->dst, max_batch);
    A(&net->coef, max_batch);
    hipStream_t st = cpals::handle_stream(h);
    if (e == hipSuccess) e = hipMemcpyAsync(net->p, params_host, cpws::N_PARAMS * sizeof(float), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(net->m, 0, cpws::N_PARAMS * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(net->v, 0, cpws::N_PARAMS * sizeof(float), st);
    if (e == hipSuccess) e = pack_all(net, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        cp_ws_destroy(net);
        return cpals::handle_fail(h, CP_ERR_HIP, (std::string("cp_ws_create: ") + hipGetErrorString(e)).c_str());
    }
    *out = net;
    return CP_OK;
}

cp_status cp_ws_destroy(cp_ws_net net) {
    if (!net) return CP_OK;
    for (void* ptr : net->allocs) (void)hipFree(ptr);
    delete net;
    return CP_OK;
}

cp_status cp_ws_get_params(cp_handle h, cp_ws_net net, float* params_host) {
    if (!h || !net || !params_host) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null argument");
    hipStream_t st = cpals::handle_stream(h);
    WS_TRY(hipMemcpyAsync(params_host, net->p, cpws::N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    WS_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    return CP_OK;
}

cp_status cp_ws_forward(cp_handle h, cp_ws_net net, const float* x_dev, int32_t B, float* y_dev) {
    if (!h || !x_dev || !y_dev) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null argument");
    cp_status s = check_batch(h, net, B);
    if (s != CP_OK) return s;
    hipStream_t st = cpals::handle_stream(h);
    const int64_t tot = (int64_t)B * net->n * 8;
    hipLaunchKernelGGL(cpws::pack_input, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x_dev, B, net->n, net->act[0]);
    WS_TRY(hipGetLastError(), "pack_input");
    WS_TRY(forward_all(net, B, st), "forward");
    WS_TRY(hipMemcpyAsync(y_dev, net->y, (size_t)B * net->n * sizeof(float), hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    return CP_OK;
}

cp_status cp_ws_gradients(cp_handle h, cp_ws_net net, const float* x_dev, const float* target_dev, int32_t B,
                          float* grad_dev, float* loss_host) {
    if (!h || !x_dev || !target_dev || !grad_dev) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null argument");
    cp_status s = check_batch(h, net, B);
    if (s != CP_OK) return s;
    if (net->n > 256) return cpals::handle_fail(h, CP_ERR_UNSUPPORTED, "training needs n <= 256");
    hipStream_t st = cpals::handle_stream(h);
    const int64_t tot = (int64_t)B * net->n * 8;
    hipLaunchKernelGGL(cpws::pack_input, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x_dev, B, net->n, net->act[0]);
    WS_TRY(hipGetLastError(), "pack_input");
    WS_TRY(forward_all(net, B, st), "forward");
    int nblk = 0;
    WS_TRY(backward_all(net, target_dev, B, st, &nblk), "backward");
    WS_TRY(hipMemcpyAsync(grad_dev, net->grad, cpws::N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    return read_loss(h, net, nblk, (int64_t)B * net->n, loss_host);
}

cp_status cp_ws_train_step(cp_handle h, cp_ws_net net, const double* traj_dev, int32_t T, int32_t C,
                           const int32_t* samples_host, const double* coef_host, int32_t B, float lr, float* loss_host) {
    if (!h || !traj_dev || !samples_host || !coef_host) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null argument");
    cp_status s = check_batch(h, net, B);
    if (s != CP_OK) return s;
    if (net->n > 256) return cpals::handle_fail(h, CP_ERR_UNSUPPORTED, "training needs n <= 256");
    if (T < 3 || C < 1) return cpals::handle_fail(h, CP_ERR_SHAPE, "need T >= 3 time levels and C >= 1 columns");
    if (!(lr > 0.f)) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "lr must be > 0");
    const int n = net->n;
    std::vector<const double*> tab(3 * (size_t)B);
    std::vector<double> cf(B);
    for (int j = 0; j < B; ++j) {
        const int t = samples_host[2 * j], c = samples_host[2 * j + 1];
        if (t < 1 || t > T - 2 || c < 0 || c >= C) return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "sample out of range");
        for (int q = 0; q < 3; ++q) tab[(size_t)q * B + j] = traj_dev + ((int64_t)(t - 1 + q) * C + c) * n;
        cf[j] = coef_host[c];
    }
    hipStream_t st = cpals::handle_stream(h);
    WS_TRY(hipMemcpyAsync(net->tab, tab.data(), tab.size() * sizeof(void*), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    WS_TRY(hipMemcpyAsync(net->coef, cf.data(), B * sizeof(double), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    hipLaunchKernelGGL(cpws::make_samples, dim3(B), dim3(cpws::TPB), 0, st, net->tab, net->tab + B, net->tab + 2 * B, net->coef, n,
                       net->act[0], net->target, net->scale);
    WS_TRY(hipGetLastError(), "make_samples");
    WS_TRY(forward_all(net, B, st), "forward");
    int nblk = 0;
    WS_TRY(backward_all(net, net->target, B, st, &nblk), "backward");
    net->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)net->t), c2 = 1.f - powf(b2, (float)net->t);
    hipLaunchKernelGGL(cpws::adam_update, dim3(ceil_div(cpws::N_PARAMS, 256)), dim3(256), 0, st, net->p, net->m, net->v, net->grad,
                       cpws::N_PARAMS, lr, b1, b2, 1e-8f, c1, c2);
    WS_TRY(hipGetLastError(), "adam_update");
    WS_TRY(pack_all(net, st), "pack_weights");
    return read_loss(h, net, nblk, (int64_t)B * n, loss_host);
}

cp_status cp_ws_predict(cp_handle h, cp_ws_net net, const cp_tensor* f_prev, const cp_tensor* f_cur, const double* coef_host,
                        cp_tensor* f_guess) {
    if (!h || !net || !f_prev || !f_cur || !coef_host || !f_guess)
        return cpals::handle_fail(h, CP_ERR_INVALID_ARG, "null argument");
    cp_status s;
    if ((s = cpals::handle_check_tensor(h, f_prev, "f_prev")) != CP_OK) return s;
    if ((s = cpals::handle_check_tensor(h, f_cur, "f_cur")) != CP_OK) return s;
    if ((s = cpals::handle_check_tensor(h, f_guess, "f_guess")) != CP_OK) return s;
    const int d = f_cur->d, r = f_cur->r;
    if (f_prev->d != d || f_guess->d != d || f_prev->r != r || f_guess->r != r)
        return cpals::handle_fail(h, CP_ERR_SHAPE, "f_prev, f_cur and f_guess must have the same dimension and rank");
    for (int k = 0; k < d; ++k)
        if (f_prev->n[k] != net->n || f_cur->n[k] != net->n || f_guess->n[k] != net->n)
            return cpals::handle_fail(h, CP_ERR_SHAPE, "every n_k must equal the network's n");
    const int B = d * r;
    if ((s = check_batch(h, net, B)) != CP_OK) return s;
    std::vector<const double*> tab(2 * (size_t)B);
    std::vector<double*> dst(B);
    std::vector<double> cf(B);
    for (int k = 0; k < d; ++k)
        for (int l = 0; l < r; ++l) {
            const int j = k * r + l;
            tab[j] = f_prev->U[k] + (int64_t)l * f_prev->ld[k];
            tab[B + j] = f_cur->U[k] + (int64_t)l * f_cur->ld[k];
            dst[j] = f_guess->U[k] + (int64_t)l * f_guess->ld[k];
            cf[j] = coef_host[k];
        }
    hipStream_t st = cpals::handle_stream(h);
    WS_TRY(hipMemcpyAsync(net->tab, tab.data(), tab.size() * sizeof(void*), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    WS_TRY(hipMemcpyAsync(net->dst, dst.data(), dst.size() * sizeof(void*), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    WS_TRY(hipMemcpyAsync(net->coef, cf.data(), B * sizeof(double), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    hipLaunchKernelGGL(cpws::make_samples, dim3(B), dim3(cpws::TPB), 0, st, net->tab, net->tab + B, (const double* const*)nullptr,
                       net->coef, net->n, net->act[0], (float*)nullptr, net->scale);
    WS_TRY(hipGetLastError(), "make_samples");
    WS_TRY(forward_all(net, B, st), "forward");
    const int64_t tot = (int64_t)B * net->n;
    hipLaunchKernelGGL(cpws::finish_guess, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, net->tab,
                       net->tab + B, (double* const*)net->dst, net->scale, net->y, net->n, B);
    WS_TRY(hipGetLastError(), "finish_guess");
    // the host tables must outlive the asynchronous copies
    WS_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    return CP_OK;
}

}  // extern "C"
