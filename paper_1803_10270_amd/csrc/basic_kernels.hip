// Streaming CP primitives on gfx950: scalar products of CP tensors (Section 2.2) and
// application of a separable operator (Section 3.2).  These are HBM-bound: each factor
// panel is read once from HBM.
#include <hip/hip_runtime.h>
#include "cpals_internal.h"

namespace cpals {

constexpr int GT = 256;       // threads per workgroup for the streaming kernels
constexpr int GROWS = 256;    // rows per workgroup chunk of a Gram partial


// One workgroup per (dimension, row chunk): partial[chunk][l + l' * rx] = sum_rows X[i,l] Y[i,l'].
// Rows are staged through LDS (coalesced HBM reads), each thread owns a few (l, l') entries.
__global__ void __launch_bounds__(GT) gram_partials(GramJob job, double* __restrict__ partial) {
    constexpr int TR = 32;
    __shared__ double xs[TR][CP_MAX_RANK + 1];
    __shared__ double ys[TR][CP_MAX_RANK + 1];
    const int c = blockIdx.x;
    int k = 0;
    while (k + 1 < job.d && c >= job.chunk0[k + 1]) ++k;
    const int row0 = (c - job.chunk0[k]) * GROWS;
    const int n = job.n[k], rx = job.rx, ry = job.ry;
    const int row1 = min(n, row0 + GROWS);
    const double* X = job.X[k];
    const double* Y = job.Y[k];
    const int ne = rx * ry;
    double acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0;
    for (int rb = row0; rb < row1; rb += TR) {
        const int nrow = min(TR, row1 - rb);
        __syncthreads();
        for (int t = threadIdx.x; t < TR * rx; t += GT) {
            const int i = t % TR, l = t / TR;
            xs[i][l] = (i < nrow) ? X[(rb + i) + (int64_t)l * job.ldx[k]] : 0.0;
        }
        for (int t = threadIdx.x; t < TR * ry; t += GT) {
            const int i = t % TR, l = t / TR;
            ys[i][l] = (i < nrow) ? Y[(rb + i) + (int64_t)l * job.ldy[k]] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = threadIdx.x + e * GT;
            if (t < ne) {
                const int l = t % rx, lp = t / rx;
                double a = acc[e];
                for (int i = 0; i < nrow; ++i) a = fma(xs[i][l], ys[i][lp], a);
                acc[e] = a;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = threadIdx.x + e * GT;
        if (t < ne) partial[(int64_t)c * ne + t] = acc[e];
    }
}

// One workgroup: Gram_k = sum of chunk partials (fixed order), out = sum_{l,l'} prod_k Gram_k.
__global__ void __launch_bounds__(GT) gram_finish(GramJob job, const double* __restrict__ partial, double* out,
                                                  int sqrt_out) {
    __shared__ double red[GT / 64];
    const int ne = job.rx * job.ry;
    double part = 0.0;
    for (int t = threadIdx.x; t < ne; t += GT) {
        double prod = 1.0;
        for (int k = 0; k < job.d; ++k) {
            double g = 0.0;
            for (int c = job.chunk0[k]; c < job.chunk0[k + 1]; ++c) g += partial[(int64_t)c * ne + t];
            prod *= g;
        }
        part += prod;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < GT / 64; ++w) s += red[w];
        *out = sqrt_out ? sqrt(fmax(s, 0.0)) : s;
    }
}

int gram_chunks(const int32_t* n, int d, int32_t* chunk0) {
    chunk0[0] = 0;
    for (int k = 0; k < d; ++k) chunk0[k + 1] = chunk0[k] + (n[k] + GROWS - 1) / GROWS;
    return chunk0[d];
}

hipError_t launch_inner(const GramJob& job, double* partial, double* out, bool sqrt_out, hipStream_t st) {
    const int nchunks = job.chunk0[job.d];
    if (nchunks > 0) hipLaunchKernelGGL(gram_partials, dim3(nchunks), dim3(GT), 0, st, job, partial);
    hipLaunchKernelGGL(gram_finish, dim3(1), dim3(GT), 0, st, job, partial, out, sqrt_out ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// operator application: Y_k[:, e*r + l] = (k == 0 ? coef_e : 1) * E_k^e X_k[:, l]
// ------------------------------------------------------------------------------------

// grid: (d * n_terms * r) columns x row blocks.  Rank-1 operators reduce w^T x first.
__global__ void __launch_bounds__(GT) apply_columns(ApplyJob job) {
    __shared__ double red[GT / 64];
    __shared__ double dot_s;
    const int col = blockIdx.x;
    const int k = col / (job.n_terms * job.r);
    const int rem = col % (job.n_terms * job.r);
    const int e = rem / job.r, l = rem % job.r;
    const int n = job.n[k];
    const OpDev op = job.ops[k][job.op_index[e * job.d + k]];
    const double scale = (k == 0) ? job.coef[e] : 1.0;
    const double* x = job.X[k] + (int64_t)l * job.ldx[k];
    double* y = job.Y[k] + (int64_t)(e * job.r + l) * job.ldy[k];
    if (op.kind == CP_OP_RANK1) {
        double part = 0.0;
        for (int i = threadIdx.x; i < n; i += GT) part = fma(op.data[n + i], x[i], part);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < GT / 64; ++w) s += red[w];
            dot_s = s;
        }
        __syncthreads();
    }
    const int rows_per = (n + gridDim.y - 1) / gridDim.y;
    const int i0 = blockIdx.y * rows_per, i1 = min(n, i0 + rows_per);
    for (int i = i0 + threadIdx.x; i < i1; i += GT) {
        double v;
        switch (op.kind) {
            case CP_OP_IDENTITY: v = x[i]; break;
            case CP_OP_DIAG: v = op.data[i] * x[i]; break;
            case CP_OP_BAND: {
                v = 0.0;
                const int h = op.hbw;
                for (int j = 0; j <= 2 * h; ++j) {
                    int c = i + j - h;
                    c %= n;
                    if (c < 0) c += n;
                    v = fma(op.data[(int64_t)j * n + i], x[c], v);
                }
                break;
            }
            default: v = op.data[i] * dot_s; break;
        }
        y[i] = scale * v;
    }
}

hipError_t launch_apply(const ApplyJob& job, int max_n, hipStream_t st) {
    const int cols = job.d * job.n_terms * job.r;
    int rb = (max_n + 4095) / 4096;
    if (rb < 1) rb = 1;
    hipLaunchKernelGGL(apply_columns, dim3(cols, rb), dim3(GT), 0, st, job);
    return hipGetLastError();
}

}  // namespace cpals
