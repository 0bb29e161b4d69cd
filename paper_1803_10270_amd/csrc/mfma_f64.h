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
    __device__ __forceinline__ void add(int i, double x) { v[i] += x; }
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
    __device__ __forceinline__ void add(int i, double x) { v[i] += (float)x; }
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
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
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
            for (int t = tid_here(); t < PG_KCH * nw; t += WG) {
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
// Gram products over the rows i_begin .. i_end - 1, in chunks staged in LDS:
//   G1 (M1 x M1, symmetric) = A^T A  and optionally  G2 (M1 x N2) = A^T B,
// where element (i, c) of A (c < M1) and of B (c < N2) come from panel functors with
//   raw(i, c) -> raw_t (loads only) and val(raw_t) -> double,
// so that a batch of loads is issued before any value is formed.
// Only the upper-triangular tiles of G1 (row tile <= column tile) are computed; both halves
// are written unless `mirror` is off (then the tiles below the diagonal are left as they
// are).  Tiles are dealt round-robin to the waves, up to GRAM_TPW per wave per pass over the
// rows.  Chunks of 32 rows (16 when LDS is short or there are at most 16 rows) are staged;
// `lds` holds `cap` doubles, at least 16 * ((TM1*16 + 1) + (TN2*16 + 1)).  Starts and ends
// with a barrier.
// ---------------------------------------------------------------------------------------
constexpr int GRAM_TPW = 9;

// The matrix-core steps of one staged chunk for the first NT tile slots of a wave: all
// operand reads of a k-step first, then NT independent steps, none of them predicated (an
// idle slot accumulates tile (0, 0) into a tile that is never stored), so the reads are
// not sunk into branches and overlap the steps.
template <bool F32, int NT>
__device__ __forceinline__ void gram_ksteps(Tile<F32> (&acc)[GRAM_TPW], const double* As, const double* Bs, int wa,
                                            int wb, int KC, int kk, int cc, const int (&ti)[GRAM_TPW],
                                            const int (&tj)[GRAM_TPW], const int (&which)[GRAM_TPW]) {
    for (int k0 = 0; k0 < KC; k0 += 4) {
        double av[NT], bv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool g1 = which[t] != 2;
            av[t] = As[(k0 + kk) * wa + ti[t] * 16 + cc];
            bv[t] = g1 ? As[(k0 + kk) * wa + tj[t] * 16 + cc] : Bs[(k0 + kk) * wb + tj[t] * 16 + cc];
        }
        // operands swapped: the tile holds the transposed block, so a lane's results lie in
        // one row-contiguous run (coalesced stores)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t].step(bv[t], av[t]);
    }
}

// Stage rows i0 .. i0 + 2^lg - 1 of a panel functor into LDS (row stride ld), `total` =
// 2^lg * (columns rounded to 16); four elements' loads per thread are in flight together.
template <class F>
__device__ __forceinline__ void gram_stage(const F& f, int n, int i0, int ncol, int total, int lg, double* dst, int ld) {
    const int msk = (1 << lg) - 1;
    for (int t0 = tid_here(); t0 < total; t0 += 4 * WG) {
        typename F::raw_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * WG;
            const int i = i0 + (t & msk), c = t >> lg;
            v[u] = (t < total && i < n && c < ncol) ? f.raw(i, c) : F::zero();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * WG;
            if (t < total) dst[(t & msk) * ld + (t >> lg)] = f.val(v[u]);
        }
    }
}

template <bool F32, class FA, class FB>
__device__ __forceinline__ void gram_lds(int i_begin, int i_end, int M1, int N2, const FA& fa, const FB& fb,
                                         double* __restrict__ G1, int ld1, double* __restrict__ G2, int ld2, double* lds,
                                         int cap, bool mirror = true) {
    const int n = i_end;   // rows i_begin .. i_end - 1
    constexpr int PFN = 16;   // prefetched elements per thread and operand
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    const int TM = (M1 + 15) >> 4, TN = (N2 + 15) >> 4;
    const int wa = TM * 16 + 1, wb = TN * 16 + 1;   // LDS row strides (odd: bank spread)
    // chunk rows: 32 (or 16), double-buffered when the LDS area allows it; with double
    // buffering the next chunk's loads are in flight during this chunk's matrix-core work
    // (16 when there are at most 16 rows: no matrix-core steps over zero padding)
    int lgKC = (n - i_begin <= 16) ? 4 : 5;
    while (lgKC > 4 && 2 * (1 << lgKC) * (wa + wb) > cap) --lgKC;
    const bool dbl = 2 * (1 << lgKC) * (wa + wb) <= cap;
    if (!dbl && n - i_begin > 16) lgKC = (32 * (wa + wb) <= cap) ? 5 : 4;
    const int KC = 1 << lgKC;
    const int na = KC * TM * 16, nb = KC * TN * 16;
    const bool pre = dbl && na <= PFN * WG && nb <= PFN * WG;
    const int bufsz = KC * (wa + wb);
    const int nt1 = TM * (TM + 1) / 2;
    const int ntiles = nt1 + TM * TN;
    const int per_pass = NWAVES * GRAM_TPW;
    const int kk = lane >> 4, cc = lane & 15;
    const int msk = KC - 1;
    for (int base = 0; base < ntiles; base += per_pass) {
        // tile slots this pass occupies per wave (1, 2, 3, 5 or 9: one instantiation each)
        const int need = (min(per_pass, ntiles - base) + NWAVES - 1) / NWAVES;
        const int nslot = need <= 3 ? need : (need <= 5 ? 5 : GRAM_TPW);
        int ti[GRAM_TPW], tj[GRAM_TPW], which[GRAM_TPW];
#pragma unroll
        for (int t = 0; t < GRAM_TPW; ++t) {
            int id = base + wave + NWAVES * t;
            which[t] = -1;
            ti[t] = tj[t] = 0;
            if (id < nt1) {
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
        Tile<F32> acc[GRAM_TPW];
#pragma unroll
        for (int t = 0; t < GRAM_TPW; ++t) acc[t].zero();
        __syncthreads();
        gram_stage(fa, n, i_begin, M1, na, lgKC, lds, wa);
        gram_stage(fb, n, i_begin, N2, nb, lgKC, lds + KC * wa, wb);
        __syncthreads();
        for (int c = 0; i_begin + c * KC < n; ++c) {
            const int buf = pre ? (c & 1) : 0;
            const double* As = lds + buf * bufsz;
            const double* Bs = As + KC * wa;
            const int i1 = i_begin + (c + 1) * KC;
            const bool more = i1 < n;
            typename FA::raw_t ra[PFN];
            typename FB::raw_t rb[PFN];
            if (pre && more) {
#pragma unroll
                for (int u = 0; u < PFN; ++u) {
                    const int t = tid_here() + u * WG;
                    const int i = i1 + (t & msk), col = t >> lgKC;
                    ra[u] = (t < na && i < n && col < M1) ? fa.raw(i, col) : FA::zero();
                    rb[u] = (t < nb && i < n && col < N2) ? fb.raw(i, col) : FB::zero();
                }
            }
            switch (nslot) {
                case 1: gram_ksteps<F32, 1>(acc, As, Bs, wa, wb, KC, kk, cc, ti, tj, which); break;
                case 2: gram_ksteps<F32, 2>(acc, As, Bs, wa, wb, KC, kk, cc, ti, tj, which); break;
                case 3: gram_ksteps<F32, 3>(acc, As, Bs, wa, wb, KC, kk, cc, ti, tj, which); break;
                case 5: gram_ksteps<F32, 5>(acc, As, Bs, wa, wb, KC, kk, cc, ti, tj, which); break;
                default: gram_ksteps<F32, GRAM_TPW>(acc, As, Bs, wa, wb, KC, kk, cc, ti, tj, which); break;
            }
            if (!more) break;
            if (pre) {
                double* An = lds + (buf ^ 1) * bufsz;
                double* Bn = An + KC * wa;
#pragma unroll
                for (int u = 0; u < PFN; ++u) {
                    const int t = tid_here() + u * WG;
                    if (t < na) An[(t & msk) * wa + (t >> lgKC)] = fa.val(ra[u]);
                    if (t < nb) Bn[(t & msk) * wb + (t >> lgKC)] = fb.val(rb[u]);
                }
                __syncthreads();
            } else {
                __syncthreads();
                gram_stage(fa, n, i1, M1, na, lgKC, lds, wa);
                gram_stage(fb, n, i1, N2, nb, lgKC, lds + KC * wa, wb);
                __syncthreads();
            }
        }
#pragma unroll
        for (int t = 0; t < GRAM_TPW; ++t) {
            if (which[t] < 0) continue;
            const int row = ti[t] * 16 + cc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = tj[t] * 16 + Tile<F32>::row(lane, v);
                const double val = acc[t].get(v);
                if (which[t] == 1) {
                    if (row < M1 && col < M1) {
                        stg(G1 + row + (int64_t)col * ld1, val);
                        // mirror into the lower triangle (diagonal tiles hold both halves)
                        if (mirror && ti[t] != tj[t]) stg(G1 + col + (int64_t)row * ld1, val);
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
