// Device helpers for the persistent CP-ALS workgroup: reductions, 1-D operator
// application, and workgroup-level FP64 contractions.
#pragma once
#include <hip/hip_runtime.h>
#include "cpals_internal.h"

namespace cpals {

// Loads and stores of device (global) memory.  Pointers reach the kernels through
// descriptors, so the compiler cannot prove their address space by itself; without these
// casts every access would become a FLAT instruction, whose completion also gates the
// LDS wait counter.
typedef const double __attribute__((address_space(1)))* gcdp;
typedef double __attribute__((address_space(1)))* gdp;
__device__ __forceinline__ double ldg(const double* p) { return *(gcdp)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(gdp)p = v; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;  // valid in lane 0
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// threadIdx.x through an opaque move: index arithmetic derived from it is recomputed where
// it is used instead of being hoisted out of the persistent loops (where it would occupy
// registers for the whole kernel).
__device__ __forceinline__ int tid_here() {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

// Batched element loop over t < total (grid-stride over the workgroup): U loads are issued
// before any result is consumed, so their latencies overlap.  ld(t) -> value, st(t, value).
template <int U, class LD, class ST>
__device__ __forceinline__ void batched_loop(int total, const LD& ld, const ST& st) {
    for (int t0 = tid_here(); t0 < total; t0 += U * WG) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            v[u] = (t < total) ? ld(t) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            if (t < total) st(t, v[u]);
        }
    }
}

// floor(t / den) for 0 <= t < 2^21, den >= 1, through a float reciprocal inv ~ 1/den
// (exact in that range: the relative error of the product stays below 2^-22).
__device__ __forceinline__ int fdiv(int t, float inv) { return (int)(((float)t + 0.5f) * inv); }

// Sum of one value per thread over the workgroup; every thread gets the result.
// `red` is an LDS array of at least NWAVES doubles.  Fixed reduction tree (deterministic).
__device__ __forceinline__ double wg_sum(double v, double* red) {
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NWAVES; ++i) s += red[i];
    return s;
}

// Two sums at once.
__device__ __forceinline__ void wg_sum2(double& a, double& b, double* red) {
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    __syncthreads();
    if (lane == 0) { red[wave] = a; red[NWAVES + wave] = b; }
    __syncthreads();
    double s = 0.0, t = 0.0;
#pragma unroll
    for (int i = 0; i < NWAVES; ++i) { s += red[i]; t += red[NWAVES + i]; }
    a = s;
    b = t;
}

// out[l] = sum_i a[i] * B[i + l*ldb], l < ncol (one wave per column, rows strided by lane).
// Result in LDS `out`.  Ends with a barrier.
__device__ __forceinline__ void wg_coldots(int n, int ncol, const double* a, const double* B, int ldb, double* out) {
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    for (int l = wave; l < ncol; l += NWAVES) {
        double s = 0.0;
        for (int i = lane; i < n; i += 64) s = fma(ldg(a + i), B[i + (int64_t)l * ldb], s);
        s = wave_sum(s);
        if (lane == 0) out[l] = s;
    }
    __syncthreads();
}

// y = O x for an n x r panel (column-major, ld = n for both).  For a rank-1 operator
// O = m w^T, `dots` must hold w^T x[:, l] (computed beforehand).  Grid-stride over the
// workgroup; no barrier.
__device__ __forceinline__ void apply_op(const OpDev& op, int n, int r, const double* x, int ldx,
                                         double* y, int ldy, const double* dots) {
    const int total = n * r;
    for (int t = tid_here(); t < total; t += WG) {
        const int i = t % n, l = t / n;
        const double* xc = x + (int64_t)l * ldx;
        double v;
        switch (op.kind) {
            case CP_OP_IDENTITY: v = ldg(xc + i); break;
            case CP_OP_DIAG: v = ldg(op.data + i) * ldg(xc + i); break;
            case CP_OP_BAND: {
                v = 0.0;
                const int h = op.hbw;
                for (int j = 0; j <= 2 * h; ++j) {
                    int c = i + j - h;
                    c %= n;
                    if (c < 0) c += n;
                    v = fma(ldg(op.data + j * n + i), ldg(xc + c), v);
                }
                break;
            }
            default: v = ldg(op.data + i) * dots[l]; break;  // rank-1: m[i] * (w^T x_l)
        }
        stg(y + i + (int64_t)l * ldy, v);
    }
}

// y (+)= O^T z.  For rank-1 O = m w^T, O^T z = w (m^T z): `dots` must hold m^T z[:, l].
template <bool ACC>
__device__ __forceinline__ void apply_op_t(const OpDev& op, int n, int r, const double* z, int ldz,
                                           double* y, int ldy, const double* dots) {
    const int total = n * r;
    for (int t = tid_here(); t < total; t += WG) {
        const int i = t % n, l = t / n;
        const double* zc = z + (int64_t)l * ldz;
        double v;
        switch (op.kind) {
            case CP_OP_IDENTITY: v = zc[i]; break;
            case CP_OP_DIAG: v = op.data[i] * zc[i]; break;
            case CP_OP_BAND: {
                // (O^T z)[i] = sum_j O[k, i] z[k] with k = i - j + h (mod n), O[k, i] = data[j][k]
                v = 0.0;
                const int h = op.hbw;
                for (int j = 0; j <= 2 * h; ++j) {
                    int k = i - j + h;
                    k %= n;
                    if (k < 0) k += n;
                    v = fma(op.data[j * n + k], zc[k], v);
                }
                break;
            }
            default: v = op.data[n + i] * dots[l]; break;  // rank-1 transpose: w[i] * (m^T z_l)
        }
        double* yp = y + i + (int64_t)l * ldy;
        if (ACC) *yp += v; else *yp = v;
    }
}

}  // namespace cpals
