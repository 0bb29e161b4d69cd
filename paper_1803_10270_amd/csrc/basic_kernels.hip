// Streaming CP primitives on gfx950: scalar products of CP tensors (Section 2.2) and
// application of a separable operator (Section 3.2).  These are HBM-bound: each factor
// panel is read once from HBM.
#include <hip/hip_runtime.h>
#include <mutex>
#include "cpals_internal.h"
#include "mfma_f64.h"

namespace cpals {

constexpr int GT = 256;       // threads per workgroup for the streaming kernels
constexpr int GTR = 64;       // rows per staged tile of a Gram partial
constexpr int MAX_CHUNKS = 2048;   // row chunks over all dimensions (bounds the final sum)

// One workgroup per (dimension, row chunk): partial[chunk][l + l' * rx] = sum_rows X[i,l] Y[i,l'].
// Tiles of 64 rows of both panels are staged through LDS (dynamic size 2 * 64 (RP + 1)
// doubles, RP = both ranks rounded up to 16, 32 or 64; each column's 64 rows are one
// contiguous 512-byte read, columns past the rank are staged as zeros).  The next tile's
// loads are issued into registers before the current tile is contracted.  The contraction
// runs on the FP64 matrix cores: wave w takes rows 16w .. 16w + 15 of the tile (four
// 16x16x4 steps) for every 16 x 16 block of the Gram; the four waves' blocks are added in
// wave order once per chunk.
template <int RP>
__global__ void __launch_bounds__(GT, RP <= 32 ? 2 : 1) gram_partials(GramJob job, double* __restrict__ partial) {
    extern __shared__ double gsm[];
    constexpr int S = RP + 1;          // LDS row stride (odd: spreads the banks)
    constexpr int U = GTR * RP / GT;   // staged elements per thread and panel
    constexpr int NT = RP / 16;        // 16-column blocks per panel at most
    static_assert(GTR == 16 * (GT / 64), "each wave contracts 16 rows of a tile");
    const int c = blockIdx.x;
    int k = 0;
    while (k + 1 < job.d && c >= job.chunk0[k + 1]) ++k;
    const int rows = job.chunk_rows[k];
    const int row0 = (c - job.chunk0[k]) * rows;
    const int n = job.n[k], rx = job.rx, ry = job.ry;
    const int row1 = min(n, row0 + rows);
    const double* X = job.X[k];
    const double* Y = job.Y[k];
    const int64_t ldx = job.ldx[k], ldy = job.ldy[k];
    double* xs = gsm;
    double* ys = gsm + GTR * S;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, cc = lane & 15;
    const int tx = (rx + 15) >> 4, ty = (ry + 15) >> 4;
    double vx[U], vy[U];
    auto load = [&](int rb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = threadIdx.x + u * GT;
            const int i = t & (GTR - 1), l = t / GTR;
            const int row = rb + i;
            vx[u] = (l < rx && row < row1) ? X[row + (int64_t)l * ldx] : 0.0;
            vy[u] = (l < ry && row < row1) ? Y[row + (int64_t)l * ldy] : 0.0;
        }
    };
    d4 acc[NT * NT];
#pragma unroll
    for (int t = 0; t < NT * NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    if (row0 < row1) load(row0);
    for (int rb = row0; rb < row1; rb += GTR) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = threadIdx.x + u * GT;
            const int i = t & (GTR - 1), l = t / GTR;
            xs[i * S + l] = vx[u];
            ys[i * S + l] = vy[u];
        }
        __syncthreads();
        if (rb + GTR < row1) load(rb + GTR);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = 16 * wave + 4 * s + kq;
            double a[NT], b[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                a[t] = xs[i * S + 16 * t + cc];
                b[t] = ys[i * S + 16 * t + cc];
            }
#pragma unroll
            for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                for (int tj = 0; tj < NT; ++tj)
                    if (ti < tx && tj < ty) acc[ti * NT + tj] = mfma_f64(a[ti], b[tj], acc[ti * NT + tj]);
        }
    }
    // block (ti, tj), element v of a lane: Gram[16 ti + kq + 4 v][16 tj + cc]
    const int ne = rx * ry;
#pragma unroll
    for (int t = 0; t < NT * NT; ++t) {
        const int ti = t / NT, tj = t % NT;
        if (ti >= tx || tj >= ty) continue;
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) gsm[(wave * 4 + v) * 64 + lane] = acc[t][v];
        __syncthreads();
        const int v = threadIdx.x >> 6;
        double sum = gsm[v * 64 + lane];
#pragma unroll
        for (int w = 1; w < GT / 64; ++w) sum += gsm[(w * 4 + v) * 64 + lane];
        const int l = 16 * ti + kq + 4 * v, lp = 16 * tj + cc;
        if (l < rx && lp < ry) partial[(int64_t)c * ne + l + lp * rx] = sum;
    }
}

// Gram_k[e] = sum over the dimension's chunk partials, one workgroup per entry e and
// dimension k (each thread adds a strided share, then a fixed reduction tree), written after
// the partials at gram[k * ne + e].
__global__ void __launch_bounds__(GT) gram_reduce(GramJob job, const double* __restrict__ partial,
                                                  double* __restrict__ gram) {
    __shared__ double red[GT / 64];
    const int ne = job.rx * job.ry;
    const int e = blockIdx.x, k = blockIdx.y;
    double g = 0.0;
    for (int c = job.chunk0[k] + threadIdx.x; c < job.chunk0[k + 1]; c += GT) g += partial[(int64_t)c * ne + e];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) g += __shfl_down(g, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s2 = 0.0;
        for (int w = 0; w < GT / 64; ++w) s2 += red[w];
        gram[(int64_t)k * ne + e] = s2;
    }
}

// One workgroup: out = sum_{l,l'} prod_k Gram_k[l, l'] (sqrt for the norm).
__global__ void __launch_bounds__(GT) gram_finish(GramJob job, const double* __restrict__ gram, double* out,
                                                  int sqrt_out) {
    __shared__ double red[GT / 64];
    const int ne = job.rx * job.ry;
    double part = 0.0;
    for (int t = threadIdx.x; t < ne; t += GT) {
        double prod = 1.0;
        for (int k = 0; k < job.d; ++k) prod *= gram[(int64_t)k * ne + t];
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

// Row chunks per dimension: at least 256 rows each, and no more than MAX_CHUNKS / d chunks
// per dimension (long panels get longer chunks).
int gram_chunks(const int32_t* n, int d, int32_t* chunk0, int32_t* chunk_rows, int max_chunks) {
    chunk0[0] = 0;
    const int per_dim = (max_chunks < MAX_CHUNKS ? max_chunks : MAX_CHUNKS) / d;
    for (int k = 0; k < d; ++k) {
        int rows = 256;
        while ((n[k] + rows - 1) / rows > per_dim) rows *= 2;
        chunk_rows[k] = rows;
        chunk0[k + 1] = chunk0[k] + (n[k] + rows - 1) / rows;
    }
    return chunk0[d];
}

template <int RP>
static hipError_t launch_partials(const GramJob& job, int nchunks, double* partial, hipStream_t st) {
    const size_t smem = (size_t)2 * GTR * (RP + 1) * sizeof(double);
    if (smem > 65536) {   // rank 64 stages more than the default 64 KB
        const hipError_t e = hipFuncSetAttribute((const void*)gram_partials<RP>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(gram_partials<RP>, dim3(nchunks), dim3(GT), smem, st, job, partial);
    return hipSuccess;
}

hipError_t launch_inner(const GramJob& job, double* partial, double* out, bool sqrt_out, hipStream_t st) {
    const int nchunks = job.chunk0[job.d];
    const int rmax = job.rx > job.ry ? job.rx : job.ry;
    if (rmax > CP_MAX_RANK) return hipErrorInvalidValue;
    // the per-dimension Grams follow the chunk partials in the same buffer
    double* gram = partial + (size_t)nchunks * job.rx * job.ry;
    if (nchunks > 0) {
        const hipError_t e = rmax <= 16   ? launch_partials<16>(job, nchunks, partial, st)
                             : rmax <= 32 ? launch_partials<32>(job, nchunks, partial, st)
                                          : launch_partials<64>(job, nchunks, partial, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gram_reduce, dim3(job.rx * job.ry, job.d), dim3(GT), 0, st, job, partial, gram);
    }
    hipLaunchKernelGGL(gram_finish, dim3(1), dim3(GT), 0, st, job, gram, out, sqrt_out ? 1 : 0);
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

// Without rank-1 operators: one thread per grid row i of dimension blockIdx.y.  For every
// column l the row of X is read once (coalesced over the workgroup's rows; band taps read
// the neighbouring rows, which the neighbouring threads just loaded), every distinct
// operator of the dimension is applied once, and the n_terms output columns are written
// from those values.
__global__ void __launch_bounds__(GT) apply_rows(ApplyJob job) {
    __shared__ double coef_s[CP_MAX_TERMS];
    __shared__ int32_t op_s[CP_MAX_TERMS];
    const int k = blockIdx.y;
    const int n = job.n[k];
    const int T = job.n_terms, r = job.r;
    // the term table of this dimension, read once per workgroup
    for (int e = threadIdx.x; e < T; e += GT) {
        op_s[e] = job.op_index[e * job.d + k];
        coef_s[e] = (k == 0) ? job.coef[e] : 1.0;
    }
    __syncthreads();
    const int i = blockIdx.x * GT + threadIdx.x;
    if (i >= n) return;
    const double* __restrict__ X = job.X[k];
    double* __restrict__ Y = job.Y[k];
    const int64_t ldx = job.ldx[k], ldy = job.ldy[k];
    // per-row diagonal coefficients, loaded once for all columns
    double dg[CP_MAX_OPS];
#pragma unroll
    for (int a = 0; a < CP_MAX_OPS; ++a) dg[a] = job.ops[k][a].kind == CP_OP_DIAG ? job.ops[k][a].data[i] : 1.0;
    // LB columns' loads are issued together before any output is formed
    constexpr int LB = 4;
    for (int l0 = 0; l0 < r; l0 += LB) {
        double xv[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) xv[u] = (l0 + u < r) ? X[(int64_t)(l0 + u) * ldx + i] : 0.0;
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int l = l0 + u;
            if (l >= r) break;
            const double* x = X + (int64_t)l * ldx;
            double v[CP_MAX_OPS];
#pragma unroll
            for (int a = 0; a < CP_MAX_OPS; ++a) {
                const OpDev op = job.ops[k][a];
                double val = dg[a] * xv[u];   // identity and diagonal
                if (op.kind == CP_OP_BAND) {
                    const int h = op.hbw;
                    val = 0.0;
                    for (int j = 0; j <= 2 * h; ++j) {
                        int c = i + j - h;   // periodic; the half-bandwidth may exceed n
                        while (c < 0) c += n;
                        while (c >= n) c -= n;
                        val = fma(op.data[(int64_t)j * n + i], x[c], val);
                    }
                }
                v[a] = val;
            }
            for (int e = 0; e < T; ++e) {
                const int a = op_s[e];
                double val = v[0];
#pragma unroll
                for (int b = 1; b < CP_MAX_OPS; ++b) val = (a == b) ? v[b] : val;
                Y[(int64_t)(e * r + l) * ldy + i] = coef_s[e] * val;
            }
        }
    }
}

hipError_t launch_apply(const ApplyJob& job, int max_n, hipStream_t st) {
    bool rank1 = false;
    for (int k = 0; k < job.d; ++k)
        for (int a = 0; a < CP_MAX_OPS; ++a) rank1 = rank1 || job.ops[k][a].kind == CP_OP_RANK1;
    if (!rank1) {
        hipLaunchKernelGGL(apply_rows, dim3((max_n + GT - 1) / GT, job.d), dim3(GT), 0, st, job);
        return hipGetLastError();
    }
    const int cols = job.d * job.n_terms * job.r;
    int rb = (max_n + 4095) / 4096;
    if (rb < 1) rb = 1;
    hipLaunchKernelGGL(apply_columns, dim3(cols, rb), dim3(GT), 0, st, job);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Scratch of the allocation-free scalar product: one file-scope device array per GPU,
// reached from the host only through the address hipGetSymbolAddress gives for the
// device that is current (the array's name is not a device address in host code).
// ------------------------------------------------------------------------------------
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int MAX_DEVICES = 64;
double* scratch_ptr[MAX_DEVICES] = {nullptr};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
    static std::mutex mu;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) scratch_ptr[device] = static_cast<double*>(p);
    if (cur != device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

double* noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    return scratch_ptr[device];
}

}  // namespace cpals
