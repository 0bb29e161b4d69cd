// Workgroup-level contractions on the gfx950 matrix cores: v_mfma_f64_16x16x4 (FP64) or,
// in the mixed-precision form, v_mfma_f32_16x16x4 on operands rounded to FP32.
//
// Lane layouts of one 16x16x4 step (measured on the device): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] for both; accumulator element v of lane l is
// D[(l / 16) + 4 v][l % 16] for FP64 and D[4 (l / 16) + v][l % 16] for FP32.
#pragma once
#include <hip/hip_runtime.h>
#include "cpals_internal.h"
#include "device_common.h"

namespace cpals {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int tile_row(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int tile_col(int lane) { return lane & 15; }

typedef float f4 __attribute__((ext_vector_type(4)));

// One 16 x 16 output tile accumulated on the matrix cores.
template <bool F32>
struct Tile;

template <>
struct Tile<false> {
    d4 v;
    __device__ __forceinline__ void zero() { v = d4{0.0, 0.0, 0.0, 0.0}; }
    __device__ __forceinline__ void step(double a, double b) { v = mfma_f64(a, b, v); }
    __device__ __forceinline__ double get(int i) const { return v[i]; }
    __device__ __forceinline__ static int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct Tile<true> {
    f4 v;
    __device__ __forceinline__ void zero() { v = f4{0.0f, 0.0f, 0.0f, 0.0f}; }
    __device__ __forceinline__ void step(double a, double b) {
        v = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, v, 0, 0, 0);
    }
    __device__ __forceinline__ double get(int i) const { return (double)v[i]; }
    __device__ __forceinline__ static int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

// ---------------------------------------------------------------------------------------
// Panel product  C (M x N) = alpha * A (M x K) * B' (K x N)
//   A element (i, k) comes from the functor af(i, k) (i < M, k < K);
//   B'(k, j) = Bt[j + k * ldb]  (B' stored with N-contiguous rows).
// M is the long (grid) dimension.  B' is staged through LDS in chunks of PG_KCH rows (all
// N columns), shared by every wave.  A wave owns IPW 16-row strips x NT column tiles; the
// A fragments of a whole chunk are gathered before the matrix-core steps so that their
// loads overlap.  `lds` must hold PG_KCH * (16 * ceil(N / 16) + 1) doubles.
// Starts and ends with a barrier.
// ---------------------------------------------------------------------------------------
constexpr int PG_KCH = 32;

// Epilogue functors: called once per output element (row < M, col < N) with the product
// value; their return values are summed into the thread's result.
struct StoreEp {
    double* C;
    int ldc;
    __device__ __forceinline__ double operator()(int row, int col, double v) const {
        stg(C + row + (int64_t)col * ldc, v);
        return 0.0;
    }
};

template <bool F32, int NT, int IPW, class AF, class EP>
__device__ __forceinline__ double panel_gemm(int M, int N, int K, const AF& af, const double* __restrict__ Bt, int ldb,
                             const EP& ep, double* lds) {
    double part = 0.0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
    const int groups = (tn + NT - 1) / NT;
    const int packs = (tm + IPW - 1) / IPW;
    const int items = packs * groups;
    const int kq = lane >> 4, cc = lane & 15;
    const int nw = tn * 16;
    const int ldsw = nw + 1;
    for (int base = 0; base < items; base += NWAVES) {
        const int it = base + wave;
        const bool active = it < items;
        const int pack = active ? it % packs : 0, g = active ? it / packs : 0;
        const int jt0 = g * NT;
        const int ntl = active ? min(NT, tn - jt0) : 0;
        Tile<F32> acc[IPW][NT];
#pragma unroll
        for (int s = 0; s < IPW; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[s][t].zero();
        for (int kc0 = 0; kc0 < K; kc0 += PG_KCH) {
            const int kc = min(PG_KCH, K - kc0);
            __syncthreads();
            for (int t = threadIdx.x; t < PG_KCH * nw; t += WG) {
                const int kk = t / nw, j = t - kk * nw;
                lds[kk * ldsw + j] = (kk < kc && j < N) ? ldg(Bt + j + (int64_t)(kc0 + kk) * ldb) : 0.0;
            }
            __syncthreads();
            if (active) {
                double a[IPW][PG_KCH / 4];
#pragma unroll
                for (int s = 0; s < IPW; ++s) {
                    const int i = (pack * IPW + s) * 16 + cc;
#pragma unroll
                    for (int ks = 0; ks < PG_KCH / 4; ++ks) {
                        const int k = kc0 + 4 * ks + kq;
                        a[s][ks] = (i < M && k < K && 4 * ks < kc) ? af(i, k) : 0.0;
                    }
                }
#pragma unroll
                for (int ks = 0; ks < PG_KCH / 4; ++ks) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if (t < ntl && 4 * ks < kc) {
                            const double b = lds[(4 * ks + kq) * ldsw + (jt0 + t) * 16 + cc];
#pragma unroll
                            for (int s = 0; s < IPW; ++s) acc[s][t].step(a[s][ks], b);
                        }
                    }
                }
            }
        }
        if (active) {
#pragma unroll
            for (int s = 0; s < IPW; ++s) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (t < ntl) {
                        const int col = (jt0 + t) * 16 + cc;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = (pack * IPW + s) * 16 + Tile<F32>::row(lane, v);
                            if (row < M && col < N) part += ep(row, col, acc[s][t].get(v));
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    return part;
}

// A functor for a plain column-major panel.
struct PanelA {
    const double* A;
    int lda;
    __device__ __forceinline__ double operator()(int i, int k) const { return ldg(A + i + (int64_t)k * lda); }
};

// ---------------------------------------------------------------------------------------
// Gram products over row chunks staged in LDS:
//   G1 (M1 x M1, symmetric) = A^T A  and optionally  G2 (M1 x N2) = A^T B,
// where row i of A (M1 values) and of B (N2 values) are produced by functors
//   fa(i, c) (c < M1),  fb(i, c) (c < N2).
// LDS: `lds` must hold KC * ((TM1*16 + 1) + (TN2*16 + 1)) doubles.
// Only the upper-triangular tiles of G1 are computed; both halves are written.
// Ends with a barrier.
// ---------------------------------------------------------------------------------------
constexpr int GRAM_KC = 16;
constexpr int GRAM_TILES_PER_WAVE = 4;

template <bool F32, class FA, class FB>
__device__ __forceinline__ void gram_lds(int n, int M1, int N2, const FA& fa, const FB& fb, double* __restrict__ G1, int ld1,
                         double* __restrict__ G2, int ld2, double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int TM = (M1 + 15) >> 4, TN = (N2 + 15) >> 4;
    const int wa = TM * 16 + 1, wb = TN * 16 + 1;   // LDS row strides (odd: bank spread)
    double* As = lds;
    double* Bs = lds + GRAM_KC * wa;
    const int nt1 = TM * (TM + 1) / 2;
    const int ntiles = nt1 + TM * TN;
    const int per_pass = NWAVES * GRAM_TILES_PER_WAVE;
    const int kk = lane >> 4, cc = lane & 15;
    for (int base = 0; base < ntiles; base += per_pass) {
        // tiles of this wave in this pass: base + wave + NWAVES * t
        int ti[GRAM_TILES_PER_WAVE], tj[GRAM_TILES_PER_WAVE], which[GRAM_TILES_PER_WAVE];
#pragma unroll
        for (int t = 0; t < GRAM_TILES_PER_WAVE; ++t) {
            int id = base + wave + NWAVES * t;
            which[t] = -1;
            ti[t] = tj[t] = 0;
            if (id < nt1) {
                // upper-triangle enumeration: row a, col b >= a
                int a = 0, rem = id;
                while (rem >= TM - a) { rem -= TM - a; ++a; }
                ti[t] = a;
                tj[t] = a + rem;
                which[t] = 1;
            } else if (id < ntiles) {
                id -= nt1;
                ti[t] = id % TM;
                tj[t] = id / TM;
                which[t] = 2;
            }
        }
        Tile<F32> acc[GRAM_TILES_PER_WAVE];
#pragma unroll
        for (int t = 0; t < GRAM_TILES_PER_WAVE; ++t) acc[t].zero();
        for (int i0 = 0; i0 < n; i0 += GRAM_KC) {
            __syncthreads();
            for (int t = threadIdx.x; t < GRAM_KC * TM * 16; t += WG) {
                const int row = t % GRAM_KC, c = t / GRAM_KC;
                const int i = i0 + row;
                As[row * wa + c] = (i < n && c < M1) ? fa(i, c) : 0.0;
            }
            if (N2 > 0) {
                for (int t = threadIdx.x; t < GRAM_KC * TN * 16; t += WG) {
                    const int row = t % GRAM_KC, c = t / GRAM_KC;
                    const int i = i0 + row;
                    Bs[row * wb + c] = (i < n && c < N2) ? fb(i, c) : 0.0;
                }
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < GRAM_TILES_PER_WAVE; ++t) {
                if (which[t] > 0) {
                    const double* Bsrc = (which[t] == 1) ? As : Bs;
                    const int wbs = (which[t] == 1) ? wa : wb;
#pragma unroll
                    for (int k0 = 0; k0 < GRAM_KC; k0 += 4) {
                        const double a = As[(k0 + kk) * wa + ti[t] * 16 + cc];
                        const double b = Bsrc[(k0 + kk) * wbs + tj[t] * 16 + cc];
                        acc[t].step(a, b);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < GRAM_TILES_PER_WAVE; ++t) {
            if (which[t] < 0) continue;
            const int col = tj[t] * 16 + cc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = ti[t] * 16 + Tile<F32>::row(lane, v);
                const double val = acc[t].get(v);
                if (which[t] == 1) {
                    if (row < M1 && col < M1) {
                        stg(G1 + row + (int64_t)col * ld1, val);
                        // mirror into the lower triangle (diagonal tiles hold both halves)
                        if (ti[t] != tj[t]) stg(G1 + col + (int64_t)row * ld1, val);
                    }
                } else if (row < M1 && col < N2) {
                    stg(G2 + row + (int64_t)col * ld2, val);
                }
            }
        }
    }
    __syncthreads();
}

}  // namespace cpals
