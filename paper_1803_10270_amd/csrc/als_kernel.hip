// Persistent implicit CP-ALS kernel for gfx950: one workgroup advances one problem
// through n_steps implicit time steps, entirely on the device.
//
// Per time step (Section 3.1):  minimise ||A f_{n+1} - B f_n|| by Gauss-Seidel ALS over
// the dimensions q = 1..d (eq. sequential_min).  The normal equations of dimension q
// (eq. ALS2 with eqs. ML and MR, collocation reading E^{ez}_q = (E_q^e)^T E_q^z) are
//     sum_{a,b} (O^a)^T O^b U_q (C^{ab})^T + lambda_q U_q = sum_a (O^a)^T [sum_b Q_q[b] (D^{ab})^T]
// with O^a the distinct 1-D operators of A in dimension q (the paper's map of unique
// one-dimensional integrals), the Hadamard factors
//     C^{ab} = sum_{e,z: a(e,q)=a, a(z,q)=b} eta_e eta_z  o_{k != q} G_k[a(e,k), a(z,k)]
//     D^{ab} = sum_{e,z: a(e,q)=a, b(z,q)=b} eta_e zeta_z o_{k != q} X_k[a(e,k), b(z,k)]
// of the stacked Grams G_k = P_k^T P_k, X_k = P_k^T Q_k, P_k = [O^a U_k]_a, Q_k = [F^b V_k]_b.
//
// The (n r) x (n r) system is solved by preconditioned conjugate gradients with the
// preconditioner (H_q + lambda_q I) (x) I_n, H_q = o_{k != q} U_k^T U_k (its inverse is the
// r x r Cholesky-based solve).  For A = I + skew the preconditioned spectrum lies in
// [sigma_min(A)^2, sigma_max(A)^2], so a handful of iterations reach FP64 accuracy.
#include <hip/hip_runtime.h>
#include <math.h>
#include "device_common.h"
#include "mfma_f64.h"

namespace cpals {

constexpr int SCRATCH = 15616;   // doubles of LDS shared by the phases of one dimension update
constexpr int LDS_PAIRS = 384;   // pair records of one dimension kept in LDS during assembly
constexpr int MAX_ITEMS = 48;    // work items of one Hadamard pass

struct StageSlot {               // one staged Gram block of the assembly
    int64_t base;                // element offset of entry (0, 0) of the block
    int32_t ld;                  // its leading dimension, 0 for an empty slot
    int32_t pad;
};

struct Smem;
extern __shared__ __attribute__((aligned(16))) unsigned char cpals_smem[];

struct Smem {
    Problem pb;
    double red[2 * NWAVES];
    double dots[CP_MAX_OPS * CP_MAX_OPS * CP_MAX_RANK];
    double colnorm[CP_MAX_DIMS * CP_MAX_RANK];
    double scratch[SCRATCH];
    PairRec pairs[LDS_PAIRS];
    StageSlot slots[(CP_MAX_DIMS - 1) * CP_MAX_OPS * CP_MAX_OPS];
    int32_t items[MAX_ITEMS][3];
    int32_t blk_item[CP_MAX_OPS * CP_MAX_OPS + 1];
    int32_t iscal[8];
};

// The workgroup's LDS state, reached through the LDS symbol itself so that every access
// compiles to LDS instructions, also inside non-inlined functions.
#define SMEM (*reinterpret_cast<Smem*>(cpals_smem))


// Row index i + o of a periodic grid of n points, for |o| small (one or two wraps).
__device__ __forceinline__ int wrap_idx(int i, int n) {
    if (i < 0) {
        i += n;
        while (i < 0) i += n;
    } else if (i >= n) {
        i -= n;
        while (i >= n) i -= n;
    }
    return i;
}

// Value of (O x)[i] for one 1-D operator and one column x (ld irrelevant).  For a rank-1
// operator O = m w^T, `dot` must hold w^T x.
// x is a column in device memory.
__device__ __forceinline__ double op_value(const OpDev& op, int n, int i, const double* x, double dot) {
    switch (op.kind) {
        case CP_OP_IDENTITY: return ldg(x + i);
        case CP_OP_DIAG: return ldg(op.data + i) * ldg(x + i);
        case CP_OP_BAND: {
            double v = 0.0;
            const int h = op.hbw;
            for (int j = 0; j <= 2 * h; ++j) v = fma(ldg(op.data + j * n + i), ldg(x + wrap_idx(i + j - h, n)), v);
            return v;
        }
        default: return ldg(op.data + i) * dot;
    }
}

// Element (i, c) of the stacked applied panel [O^0 X, O^1 X, ...] (column c = a*r + l).
// For a rank-1 operator O^a = m w^T, dots[a*r + l] must hold w^T X[:, l].
struct OpApplyF {
    const OpDev* ops;
    int n, r;
    const double* X;
    const double* dots;
    __device__ __forceinline__ double operator()(int i, int c) const {
        // c / r through a float reciprocal (exact for c < 2^16, r <= 64)
        const int a = (int)(((float)c + 0.5f) * __frcp_rn((float)r));
        const int l = c - a * r;
        return op_value(ops[a], n, i, X + (int64_t)l * n, dots[a * r + l]);
    }
};

// Plain column-major panel element (i, c).
struct ColF {
    const double* X;
    int ld;
    __device__ __forceinline__ double operator()(int i, int c) const { return ldg(X + i + (int64_t)c * ld); }
};

// x - u elementwise (the increment of one factor).
struct DiffF {
    const double* x;
    const double* u;
    int ld;
    __device__ __forceinline__ double operator()(int i, int c) const {
        const int64_t o = i + (int64_t)c * ld;
        return ldg(x + o) - ldg(u + o);
    }
};

// w^T X[:, l] for every rank-1 operator among ops[0..m) -> s.dots[a*r + l].  Uniform; ends
// with a barrier when there is any rank-1 operator.
__device__ __forceinline__ void rank1_dots_fwd(const OpDev* ops, int m, int n, int r, const double* X) {
    Smem& s = SMEM;
    for (int a = 0; a < m; ++a)
        if (ops[a].kind == CP_OP_RANK1) wg_coldots(n, r, ops[a].data + n, X, n, s.dots + a * r);
}

// ------------------------------------------------------------------------------------
// applied panels
// ------------------------------------------------------------------------------------

// out[:, a*r:(a+1)*r] = O^a in (n x r panel, ld ldin), for the m operators ops[0..m).
__device__ __forceinline__ void apply_ops_fwd(const OpDev* ops, int m, int n, int r, const double* in, int ldin,
                              double* out) {
    Smem& s = SMEM;
    bool any_rank1 = false;
    for (int a = 0; a < m; ++a) any_rank1 |= (ops[a].kind == CP_OP_RANK1);
    if (any_rank1) {
        for (int a = 0; a < m; ++a)
            if (ops[a].kind == CP_OP_RANK1) wg_coldots(n, r, ops[a].data + n, in, ldin, s.dots + a * r);
    }
    for (int a = 0; a < m; ++a) apply_op(ops[a], n, r, in, ldin, out + (int64_t)a * r * n, n, s.dots + a * r);
    __syncthreads();
}

// w = sum_a (O^a)^T Z[:, a-block] + lam * p ; returns <p, w> (all threads).
__device__ __forceinline__ double apply_ops_t_sum(const OpDev* ops, int m, int n, int r, const double* Z,
                                  double lam, const double* p, double* w) {
    Smem& s = SMEM;
    bool any_rank1 = false;
    for (int a = 0; a < m; ++a) any_rank1 |= (ops[a].kind == CP_OP_RANK1);
    if (any_rank1) {
        for (int a = 0; a < m; ++a)
            if (ops[a].kind == CP_OP_RANK1)
                wg_coldots(n, r, ops[a].data, Z + (int64_t)a * r * n, n, s.dots + a * r);
    }
    double part = 0.0;
    const int total = n * r;
    for (int t = threadIdx.x; t < total; t += WG) {
        const int i = t % n, l = t / n;
        const double pv = p ? p[t] : 0.0;
        double v = lam * pv;
        for (int a = 0; a < m; ++a) {
            const OpDev& op = ops[a];
            const double* zc = Z + (int64_t)a * r * n + (int64_t)l * n;
            switch (op.kind) {
                case CP_OP_IDENTITY: v += zc[i]; break;
                case CP_OP_DIAG: v = fma(op.data[i], zc[i], v); break;
                case CP_OP_BAND: {
                    const int h = op.hbw;
                    for (int j = 0; j <= 2 * h; ++j) {
                        int k = i - j + h;
                        k %= n;
                        if (k < 0) k += n;
                        v = fma(op.data[j * n + k], zc[k], v);
                    }
                    break;
                }
                default: v = fma(op.data[n + i], s.dots[a * r + l], v); break;
            }
        }
        w[t] = v;
        part = fma(pv, v, part);
    }
    return wg_sum(part, s.red);
}

// ------------------------------------------------------------------------------------
// Gram refresh of one dimension: G_k = P_k^T P_k, X_k = P_k^T Q_k with P_k = [O^a U_k]_a
// formed row chunk by row chunk in LDS (never stored).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void refresh_dim(int k, int r0, bool lowp) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[k], r = pb.r, m = pb.mA[k], mb = pb.mB[k];
    const double* Uk = pb.U + pb.offU[k];
    rank1_dots_fwd(pb.opA[k], m, n, r, Uk);
    OpApplyF fa{pb.opA[k], n, r, Uk, s.dots};
    ColF fb{pb.Q + pb.offQ[k], n};
    if (lowp) gram_lds<true>(n, m * r, mb * r0, fa, fb, pb.G + pb.offG[k], m * r, pb.X + pb.offX[k], m * r, s.scratch);
    else gram_lds<false>(n, m * r, mb * r0, fa, fb, pb.G + pb.offG[k], m * r, pb.X + pb.offX[k], m * r, s.scratch);
}

__device__ __forceinline__ void compute_Q(int k, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[k];
    apply_ops_fwd(pb.opB[k], pb.mB[k], n, r0, pb.V + pb.offV[k], n, pb.Q + pb.offQ[k]);
}

// ------------------------------------------------------------------------------------
// Hadamard assembly for dimension q: C (mA x mA blocks r x r), D (mA x mB blocks r x r0),
// H0 = o_{k != q} U_k^T U_k.  Returns trace(M_q) (without the shift).
// The Gram entries of a chunk of matrix positions are staged in LDS once (all dimensions
// k != q, all operator blocks), then eight lanes share one position and split its pair
// list; the partial sums meet through lane shuffles.
// ------------------------------------------------------------------------------------
// One Hadamard pass over the r x rc position grid of dimension q:
//   out[l + (blk rc + lc) r] = sum over the pair records of block blk of
//                              coef * prod_{j-th dim k != q} src_k[block slot_j][l, lc]
// (src = G for the C blocks, X for the D blocks).  Per chunk of E positions the entries of
// every (dimension, operator block) slot are staged in LDS; the pair list is cut into
// work items of similar length, each wave takes items and sums them for its positions
// (EPT per lane, identity-block factors held in registers), and a last pass adds the items
// of a block in a fixed order.  With WITH_H0 also H0 = prod_j src_k[slot 0] and the trace
// sum_blk trace(C^blk) <O^a, O^b>_F are produced.
template <bool WITH_H0, int EPT>
__device__ __forceinline__ double hadamard_pass(int q, int rc, int MM, const double* src, int nblk,
                                const int32_t* off, const PairRec* pairs_g, double* out, const double* trOO) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d, r = pb.r;
    const int nk = d - 1;
    const int nE = r * rc;
    constexpr int E = 64 * EPT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* st = s.scratch;
    const int p0 = off[0], np = off[nblk] - off[0];
    __syncthreads();
    const PairRec* pairs = pairs_g + p0;
    if (np <= LDS_PAIRS) {
        for (int t = threadIdx.x; t < np; t += WG) {
            const double* src_rec = reinterpret_cast<const double*>(pairs_g + p0 + t);
            double* dst_rec = reinterpret_cast<double*>(s.pairs + t);
            dst_rec[0] = ldg(src_rec);
            dst_rec[1] = ldg(src_rec + 1);
        }
        pairs = s.pairs;
    }
    for (int t = threadIdx.x; t < nk * MM; t += WG) {
        const int j = t / MM, ab = t % MM;
        const int k = j < q ? j : j + 1;
        const int mk = pb.mA[k];
        const int nb = WITH_H0 ? mk : pb.mB[k];
        StageSlot sl;
        sl.pad = 0;
        if (ab < mk * nb) {
            const int a = ab % mk, b = ab / mk;
            sl.ld = mk * r;
            sl.base = (WITH_H0 ? pb.offG[k] : pb.offX[k]) + (int64_t)(b * rc) * sl.ld + a * r;
        } else {
            sl.ld = 0;
            sl.base = 0;
        }
        s.slots[t] = sl;
    }
    if (threadIdx.x == 0) {
        int S = max(1, (np + 2 * NWAVES - 1) / (2 * NWAVES));
        int cnt;
        for (;;) {
            cnt = 0;
            for (int blk = 0; blk < nblk; ++blk) cnt += max(1, (off[blk + 1] - off[blk] + S - 1) / S);
            if (cnt <= MAX_ITEMS) break;
            S *= 2;
        }
        cnt = 0;
        for (int blk = 0; blk < nblk; ++blk) {
            s.blk_item[blk] = cnt;
            const int b0 = off[blk] - p0, b1 = off[blk + 1] - p0;
            int a = b0;
            do {
                const int e = min(b1, a + S);
                s.items[cnt][0] = blk;
                s.items[cnt][1] = a;
                s.items[cnt][2] = e;
                ++cnt;
                a = e;
            } while (a < b1);
        }
        s.blk_item[nblk] = cnt;
        s.iscal[1] = cnt;
    }
    __syncthreads();
    const int nitems = s.iscal[1];
    double* part = st + nk * MM * E;
    double trpart = 0.0;
    for (int e0 = 0; e0 < nE; e0 += E) {
        // stage the slot entries of positions e0 .. e0 + E
        {
            const int e = threadIdx.x & (E - 1);
            const int pos = e0 + e;
            const bool ok = pos < nE;
            const int l = ok ? pos % r : 0, lc = ok ? pos / r : 0;
            for (int sl = threadIdx.x / E; sl < nk * MM; sl += WG / E) {
                const StageSlot ss = s.slots[sl];
                st[sl * E + e] = (ok && ss.ld) ? ldg(src + ss.base + (int64_t)lc * ss.ld + l) : 0.0;
            }
        }
        __syncthreads();
        // identity-block factors of this lane's positions
        double h0r[CP_MAX_DIMS - 1][EPT];
#pragma unroll
        for (int j = 0; j < CP_MAX_DIMS - 1; ++j)
#pragma unroll
            for (int u = 0; u < EPT; ++u) h0r[j][u] = (j < nk) ? st[(j * MM) * E + lane + 64 * u] : 1.0;
        if (WITH_H0 && wave == 0) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int pos = e0 + lane + 64 * u;
                double prod = 1.0;
#pragma unroll
                for (int j = 0; j < CP_MAX_DIMS - 1; ++j) prod *= h0r[j][u];
                if (pos < nE) stg(pb.H0 + pos, prod);
            }
        }
        for (int it = wave; it < nitems; it += NWAVES) {
            const int i0 = s.items[it][1], i1 = s.items[it][2];
            double acc[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) acc[u] = 0.0;
            for (int pi = i0; pi < i1; ++pi) {
                const double coef = pairs[pi].coef;
                const uint64_t sw = *reinterpret_cast<const uint64_t*>(pairs[pi].slot);
                double prod[EPT];
#pragma unroll
                for (int u = 0; u < EPT; ++u) prod[u] = coef;
#pragma unroll
                for (int j = 0; j < CP_MAX_DIMS - 1; ++j) {
                    if (j < nk) {
                        const int sj = (int)((sw >> (8 * j)) & 0xffu);
                        if (sj == 0) {
#pragma unroll
                            for (int u = 0; u < EPT; ++u) prod[u] *= h0r[j][u];
                        } else {
                            const double* row = st + (j * MM + sj) * E + lane;
#pragma unroll
                            for (int u = 0; u < EPT; ++u) prod[u] *= row[64 * u];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < EPT; ++u) acc[u] += prod[u];
            }
#pragma unroll
            for (int u = 0; u < EPT; ++u) part[it * E + lane + 64 * u] = acc[u];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nblk * E; t += WG) {
            const int blk = t / E, e = t - blk * E;
            const int pos = e0 + e;
            if (pos < nE) {
                double acc = 0.0;
                for (int it = s.blk_item[blk]; it < s.blk_item[blk + 1]; ++it) acc += part[it * E + e];
                const int l = pos % r, lc = pos / r;
                stg(out + l + (int64_t)(blk * rc + lc) * r, acc);
                if (WITH_H0 && l == lc) trpart = fma(acc, trOO[blk], trpart);
            }
        }
        __syncthreads();
    }
    return trpart;
}

__device__ __forceinline__ double assemble(int q, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d, r = pb.r, mq = pb.mA[q], mbq = pb.mB[q];
    double trpart = 0.0;
    if (d == 1) {
        // every Hadamard product over k != q is empty (all ones)
        for (int t = threadIdx.x; t < mq * mq * r * r; t += WG) {
            const int blk = t / (r * r), e = t % (r * r);
            const int l = e % r, lp = e / r;
            double acc = 0.0;
            for (int pi = pb.offC[q][blk]; pi < pb.offC[q][blk + 1]; ++pi) acc += pb.pairsC[pi].coef;
            pb.Cm[l + (int64_t)(blk * r + lp) * r] = acc;
            if (l == lp) trpart = fma(acc, pb.trOO[q][blk], trpart);
        }
        for (int t = threadIdx.x; t < mq * mbq * r * r0; t += WG) {
            const int blk = t / (r * r0), e = t % (r * r0);
            const int l = e % r, l0 = e / r;
            double acc = 0.0;
            for (int pi = pb.offD[q][blk]; pi < pb.offD[q][blk + 1]; ++pi) acc += pb.pairsD[pi].coef;
            pb.Dm[l + (int64_t)(blk * r0 + l0) * r] = acc;
        }
        for (int t = threadIdx.x; t < r * r; t += WG) pb.H0[t] = 1.0;
        return wg_sum(trpart, s.red);
    }
    const int nk = d - 1;
    // positions per chunk: as many as the LDS staging area holds (items need E doubles each)
    const int MM = pb.MMq[q], MX = pb.MXq[q];
    if ((nk * MM + MAX_ITEMS) * 256 <= SCRATCH)
        trpart = hadamard_pass<true, 4>(q, r, MM, pb.G, mq * mq, pb.offC[q], pb.pairsC, pb.Cm, pb.trOO[q]);
    else if ((nk * MM + MAX_ITEMS) * 128 <= SCRATCH)
        trpart = hadamard_pass<true, 2>(q, r, MM, pb.G, mq * mq, pb.offC[q], pb.pairsC, pb.Cm, pb.trOO[q]);
    else
        trpart = hadamard_pass<true, 1>(q, r, MM, pb.G, mq * mq, pb.offC[q], pb.pairsC, pb.Cm, pb.trOO[q]);
    if ((nk * MX + MAX_ITEMS) * 256 <= SCRATCH)
        hadamard_pass<false, 4>(q, r0, MX, pb.X, mq * mbq, pb.offD[q], pb.pairsD, pb.Dm, nullptr);
    else if ((nk * MX + MAX_ITEMS) * 128 <= SCRATCH)
        hadamard_pass<false, 2>(q, r0, MX, pb.X, mq * mbq, pb.offD[q], pb.pairsD, pb.Dm, nullptr);
    else
        hadamard_pass<false, 1>(q, r0, MX, pb.X, mq * mbq, pb.offD[q], pb.pairsD, pb.Dm, nullptr);
    return wg_sum(trpart, s.red);  // includes the barrier that publishes C, D, H0
}

// ------------------------------------------------------------------------------------
// Preconditioner: Hinv = (H0 + lam I)^{-1} by in-place Gauss-Jordan elimination on the
// diagonal pivots (H0 + lam I is symmetric positive definite), all positions of the r x r
// matrix updated in parallel, two barriers per pivot.  Returns flags.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t factor_precond(double lam) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r, rr = r * r;
    double* H = s.scratch;
    for (int t = threadIdx.x; t < rr; t += WG) {
        const int i = t % r, j = t / r;
        H[t] = ldg(pb.H0 + t) + ((i == j) ? lam : 0.0);
    }
    double dpart = 0.0;
    for (int t = threadIdx.x; t < r; t += WG) dpart = fmax(dpart, ldg(pb.H0 + t + t * r) + lam);
    dpart = wave_max(dpart);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s.red[threadIdx.x >> 6] = dpart;
    __syncthreads();
    double maxdiag = 0.0;
    for (int w = 0; w < NWAVES; ++w) maxdiag = fmax(maxdiag, s.red[w]);
    uint32_t fl = 0;
    constexpr int PER = (CP_MAX_RANK * CP_MAX_RANK + WG - 1) / WG;
    for (int p = 0; p < r; ++p) {
        double piv = H[p + p * r];
        if (!(piv > 1e-12 * maxdiag)) fl |= CP_FLAG_REGULARIZED;
        if (!(piv > 0.0)) piv = (lam > 0.0) ? lam : 1e-300;
        const double ip = 1.0 / piv;
        double nv[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = threadIdx.x + u * WG;
            nv[u] = 0.0;
            if (t < rr) {
                const int i = t % r, j = t / r;
                const double hip = H[i + p * r], hpj = H[p + j * r];
                if (i == p) nv[u] = (j == p) ? ip : hpj * ip;
                else if (j == p) nv[u] = -hip * ip;
                else nv[u] = fma(-hip * ip, hpj, H[t]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = threadIdx.x + u * WG;
            if (t < rr) H[t] = nv[u];
        }
        __syncthreads();
    }
    // symmetrise (the preconditioner of CG must be symmetric)
    for (int t = threadIdx.x; t < rr; t += WG) {
        const int i = t % r, j = t / r;
        stg(pb.Hinv + t, 0.5 * (H[t] + H[j + i * r]));
    }
    __syncthreads();
    return fl;
}

// Fast composite product for operators that are all band/diagonal/identity with half
// bandwidth <= 2 (the usual finite-difference case): X is copied to LDS once, and for
// every chunk of KCH columns of the stacked panel the (at most two) composite operators
// it touches are staged in LDS as five-tap stencils, so the panel chunk is formed from
// LDS only (no dependent device-memory loads).  Requires rc >= KCH >= 4.
template <bool F32, int SPW, class EP>
__device__ __forceinline__ double comp_gemm_fast(const OpDev* comps, int nblk, int n, int rc, const double* X,
                                              const double* Kt, int KCH, const EP& ep) {
    Smem& s = SMEM;
    const int r = s.pb.r;
    const int K = nblk * rc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, cc = lane & 15;
    const int tm = (n + 15) >> 4, tn = (r + 15) >> 4;
    const int nw = tn * 16, ldb = nw + 1, ldw = n + 1;
    double* Xs = s.scratch;
    double* Ws = Xs + ((n * rc + 1) & ~1);
    double* Bs = Ws + ((ldw * KCH + 1) & ~1);
    double* Ds = Bs + ((ldb * KCH + 1) & ~1);   // two five-tap stencils, 5 n each
    __syncthreads();
    for (int t = threadIdx.x; t < n * rc; t += WG) Xs[t] = ldg(X + t);
    Tile<F32> acc[SPW][4];
#pragma unroll
    for (int u = 0; u < SPW; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[u][t].zero();
    for (int kc0 = 0; kc0 < K; kc0 += KCH) {
        const int blk0 = kc0 / rc;
        __syncthreads();
        // stencils of the blocks touched by this chunk
        for (int t = threadIdx.x; t < 2 * 5 * n; t += WG) {
            const int which = t / (5 * n), rem = t - which * 5 * n;
            const int j = rem / n, i = rem - j * n;
            const int blk = blk0 + which;
            double v = 0.0;
            if (blk < nblk) {
                const OpDev op = comps[blk];
                if (op.kind == CP_OP_IDENTITY) v = (j == 2) ? 1.0 : 0.0;
                else if (op.kind == CP_OP_DIAG) v = (j == 2) ? ldg(op.data + i) : 0.0;
                else {
                    const int jj = j - 2 + op.hbw;   // tap j sits at offset j - 2
                    v = (jj >= 0 && jj <= 2 * op.hbw) ? ldg(op.data + jj * n + i) : 0.0;
                }
            }
            Ds[t] = v;
        }
        for (int t = threadIdx.x; t < KCH * nw; t += WG) {
            const int kk = t / nw, j = t - kk * nw;
            Bs[kk * ldb + j] = (kc0 + kk < K && j < r) ? ldg(Kt + j + (int64_t)(kc0 + kk) * r) : 0.0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < KCH * n; t += WG) {
            const int kk = t / n, i = t - kk * n;
            const int c = kc0 + kk;
            double v = 0.0;
            if (c < K) {
                const int blk = c / rc, l = c - blk * rc;
                const double* d5 = Ds + (blk - blk0) * 5 * n;
                const double* x = Xs + l * n;
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    int ci = i + j - 2;
                    ci += (ci < 0) ? n : 0;
                    ci -= (ci >= n) ? n : 0;
                    v = fma(d5[j * n + i], x[ci], v);
                }
            }
            Ws[kk * ldw + i] = v;
        }
        __syncthreads();
        for (int ks = 0; ks < KCH / 4; ++ks) {
            const int kr = 4 * ks + kq;
            double b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = (t < tn) ? Bs[kr * ldb + t * 16 + cc] : 0.0;
#pragma unroll
            for (int u = 0; u < SPW; ++u) {
                const int strip = wave + NWAVES * u;
                if (strip < tm) {
                    const int i = strip * 16 + cc;
                    const double a = (i < n) ? Ws[kr * ldw + i] : 0.0;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < tn) acc[u][t].step(a, b[t]);
                }
            }
        }
    }
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
        const int strip = wave + NWAVES * u;
        if (strip < tm) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t < tn) {
                    const int col = t * 16 + cc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = strip * 16 + Tile<F32>::row(lane, v);
                        if (row < n && col < r) part += ep(row, col, acc[u][t].get(v));
                    }
                }
            }
        }
    }
    __syncthreads();
    return part;
}

// General composite product (any operator kinds, any sizes that fit): the stacked panel
// chunk is formed from device memory, column by column.
template <bool F32, int SPW, class EP>
__device__ __forceinline__ double comp_gemm_chunked(const OpDev* comps, int n, int rc, const double* X, const double* Kt,
                                    int K, int KCH, const EP& ep) {
    Smem& s = SMEM;
    const int r = s.pb.r;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kq = lane >> 4, cc = lane & 15;
    const int tm = (n + 15) >> 4, tn = (r + 15) >> 4;
    const int nw = tn * 16, ldb = nw + 1, ldw = n + 1;
    double* Ws = s.scratch;
    double* Bs = s.scratch + ((ldw * KCH + 1) & ~1);
    const int tpc = min(WG, ((n + 63) / 64) * 64);   // threads per panel column (multiple of 64)
    const int cpp = WG / tpc;                          // columns per pass
    const int my_col = threadIdx.x / tpc, my_row = threadIdx.x - my_col * tpc;
    const float inv_rc = __frcp_rn((float)rc);
    Tile<F32> acc[SPW][4];
#pragma unroll
    for (int u = 0; u < SPW; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[u][t].zero();
    for (int kc0 = 0; kc0 < K; kc0 += KCH) {
        __syncthreads();
        // W chunk: column kk = comp_blk X[:, l] for c = kc0 + kk = blk rc + l (wave-uniform c)
        if (my_col < cpp) {
            for (int kk = my_col; kk < KCH; kk += cpp) {
                const int c = kc0 + kk;
                double* wcol = Ws + kk * ldw;
                if (c < K) {
                    const int blk = (int)(((float)c + 0.5f) * inv_rc);
                    const int l = c - blk * rc;
                    const OpDev op = comps[blk];
                    const double* x = X + (int64_t)l * n;
                    const double dot = s.dots[blk * rc + l];
                    for (int i = my_row; i < n; i += tpc) wcol[i] = op_value(op, n, i, x, dot);
                } else {
                    for (int i = my_row; i < n; i += tpc) wcol[i] = 0.0;
                }
            }
        }
        for (int t = threadIdx.x; t < KCH * nw; t += WG) {
            const int kk = t / nw, j = t - kk * nw;
            Bs[kk * ldb + j] = (kc0 + kk < K && j < r) ? ldg(Kt + j + (int64_t)(kc0 + kk) * r) : 0.0;
        }
        __syncthreads();
        for (int ks = 0; ks < KCH / 4; ++ks) {
            const int kr = 4 * ks + kq;
            double b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = (t < tn) ? Bs[kr * ldb + t * 16 + cc] : 0.0;
#pragma unroll
            for (int u = 0; u < SPW; ++u) {
                const int strip = wave + NWAVES * u;
                if (strip < tm) {
                    const int i = strip * 16 + cc;
                    const double a = (i < n) ? Ws[kr * ldw + i] : 0.0;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (t < tn) acc[u][t].step(a, b[t]);
                }
            }
        }
    }
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < SPW; ++u) {
        const int strip = wave + NWAVES * u;
        if (strip < tm) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t < tn) {
                    const int col = t * 16 + cc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = strip * 16 + Tile<F32>::row(lane, v);
                        if (row < n && col < r) part += ep(row, col, acc[u][t].get(v));
                    }
                }
            }
        }
    }
    __syncthreads();
    return part;
}

// ------------------------------------------------------------------------------------
// Composite product  out = sum_blk comp_blk X (K^blk)^T  on the matrix cores:
// the stacked panel W[:, blk rc + l] = comp_blk X[:, l] is formed chunk by chunk in LDS
// (wave-uniform columns), K^blk are the r x rc blocks of Kt (Kt[l + (blk rc + l') r]).
// ------------------------------------------------------------------------------------
template <bool F32, class EP>
__device__ __forceinline__ double comp_gemm(const OpDev* comps, int nblk, int n, int rc, const double* X,
                            const double* Kt, const EP& ep) {
    Smem& s = SMEM;
    const int r = s.pb.r;
    const int K = nblk * rc;
    const int tm = (n + 15) >> 4;
    {
        // fast path: five-tap composites, chunks of KCH <= rc columns, everything in LDS
        bool five = n >= 3 && rc >= 4 && tm <= 4 * NWAVES;
        for (int b = 0; b < nblk; ++b)
            five = five && (comps[b].kind == CP_OP_IDENTITY || comps[b].kind == CP_OP_DIAG ||
                            (comps[b].kind == CP_OP_BAND && comps[b].hbw <= 2));
        const int KCHf = min(16, rc & ~3);
        const int ldbf = ((r + 15) >> 4) * 16 + 1;
        const int need = ((n * rc + 1) & ~1) + (((n + 1) * KCHf + 1) & ~1) + ((ldbf * KCHf + 1) & ~1) + 10 * n;
        if (five && need <= SCRATCH) {
            if (tm <= NWAVES) return comp_gemm_fast<F32, 1>(comps, nblk, n, rc, X, Kt, KCHf, ep);
            if (tm <= 2 * NWAVES) return comp_gemm_fast<F32, 2>(comps, nblk, n, rc, X, Kt, KCHf, ep);
            return comp_gemm_fast<F32, 4>(comps, nblk, n, rc, X, Kt, KCHf, ep);
        }
    }
    for (int b = 0; b < nblk; ++b)
        if (comps[b].kind == CP_OP_RANK1) wg_coldots(n, rc, comps[b].data + n, X, n, s.dots + b * rc);
    const int ldb = ((r + 15) >> 4) * 16 + 1;
    int KCH = 32;
    while (KCH >= 4 && (n + 1) * KCH + 2 + KCH * ldb > SCRATCH) KCH >>= 1;
    if (KCH >= 4 && tm <= 4 * NWAVES) {
        if (tm <= NWAVES) return comp_gemm_chunked<F32, 1>(comps, n, rc, X, Kt, K, KCH, ep);
        if (tm <= 2 * NWAVES) return comp_gemm_chunked<F32, 2>(comps, n, rc, X, Kt, K, KCH, ep);
        return comp_gemm_chunked<F32, 4>(comps, n, rc, X, Kt, K, KCH, ep);
    }
    OpApplyF af{comps, n, rc, X, s.dots};
    return panel_gemm<F32, 4, 2>(n, r, K, af, Kt, r, ep, s.scratch);
}

// w = (M_q + lam I) p written to w; returns <p, w>.
struct ShiftDotEp {
    double* w;
    const double* p;
    double lam;
    int ld;
    __device__ __forceinline__ double operator()(int row, int col, double v) const {
        const int64_t o = row + (int64_t)col * ld;
        const double pv = ldg(p + o);
        const double wv = fma(lam, pv, v);
        stg(w + o, wv);
        return pv * wv;
    }
};

__device__ __forceinline__ double matvec(int q, double lam, const double* p, double* w, bool lowp) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[q], r = pb.r, m = pb.mA[q];
    const double part = lowp ? comp_gemm<true>(pb.compAA[q], m * m, n, r, p, pb.Cm, ShiftDotEp{w, p, lam, n})
                             : comp_gemm<false>(pb.compAA[q], m * m, n, r, p, pb.Cm, ShiftDotEp{w, p, lam, n});
    return wg_sum(part, s.red);
}

// z = r Hinv (each grid row times the symmetric Hinv); returns <r, z>.
struct StoreDotEp {
    double* z;
    const double* rv;
    int ld;
    __device__ __forceinline__ double operator()(int row, int col, double v) const {
        const int64_t o = row + (int64_t)col * ld;
        stg(z + o, v);
        return ldg(rv + o) * v;
    }
};

__device__ __forceinline__ double precond(int n, const double* rv, double* zv) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r;
    const double part = panel_gemm<false, 4, 2>(n, r, r, PanelA{rv, n}, pb.Hinv, r, StoreDotEp{zv, rv, n}, s.scratch);
    return wg_sum(part, s.red);
}

// ------------------------------------------------------------------------------------
// one dimension update; returns ||Delta f_q||^2 and accumulates pcg iterations / flags
// ------------------------------------------------------------------------------------
// lowp: the Gram, right-hand-side and matvec contractions on FP32 matrix cores (the
// mixed-precision form); the preconditioner, the increment and all scalars stay FP64.
__device__ __forceinline__ double update_dim(int q, int r0, int& pcg_iters, uint32_t& flags, bool lowp) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[q], r = pb.r, m = pb.mA[q], mb = pb.mB[q];
    const int nr = n * r;
    double* Uq = pb.U + pb.offU[q];

    const double trM = assemble(q, r0);
    const double lam = pb.eps_reg * trM / (double)nr;

    // right-hand side b = sum_{a,b'} (O_A^a)^T O_B^b' V_q (D^{a b'})^T
    if (lowp) comp_gemm<true>(pb.compAB[q], m * mb, n, r0, pb.V + pb.offV[q], pb.Dm, StoreEp{pb.vb, n});
    else comp_gemm<false>(pb.compAB[q], m * mb, n, r0, pb.V + pb.offV[q], pb.Dm, StoreEp{pb.vb, n});

    flags |= factor_precond(lam);

    // PCG from the current factor
    double* x = pb.vx;
    double* rv = pb.vr;
    double* z = pb.vz;
    double* p = pb.vp;
    double* w = pb.vw;
    for (int t = threadIdx.x; t < nr; t += WG) stg(x + t, ldg(Uq + t));
    __syncthreads();
    // Stopping test in the preconditioned (energy-like) norm: r^T P^{-1} r <= tol^2 b^T P^{-1} b.
    // Since P ~ J_q^T J_q, this bounds the change of the represented tensor, also along
    // near-singular directions of H_q where the plain residual norm says little.
    const double bz = precond(n, pb.vb, z);
    matvec(q, lam, x, w, lowp);
    for (int t = threadIdx.x; t < nr; t += WG) stg(rv + t, ldg(pb.vb + t) - ldg(w + t));
    __syncthreads();
    double rz = precond(n, rv, z);
    // FP32 contractions cannot resolve the system below ~1e-7; the FP64 sweeps finish it
    const double ptol = lowp ? fmax(pb.pcg_tol, 1e-6) : pb.pcg_tol;
    const double stop = ptol * ptol * bz;
    int it = 0;
    if (rz > stop) {
        for (int t = threadIdx.x; t < nr; t += WG) stg(p + t, ldg(z + t));
        __syncthreads();
        for (it = 1; it <= pb.pcg_max; ++it) {
            const double pw = matvec(q, lam, p, w, lowp);
            const double alpha = rz / pw;
            for (int t = threadIdx.x; t < nr; t += WG) {
                stg(x + t, fma(alpha, ldg(p + t), ldg(x + t)));
                stg(rv + t, fma(-alpha, ldg(w + t), ldg(rv + t)));
            }
            __syncthreads();
            const double rzn = precond(n, rv, z);
            if (rzn <= stop || !(pw > 0.0)) break;
            const double beta = rzn / rz;
            rz = rzn;
            for (int t = threadIdx.x; t < nr; t += WG) stg(p + t, fma(beta, ldg(p + t), ldg(z + t)));
            __syncthreads();
        }
        if (it > pb.pcg_max) {
            flags |= CP_FLAG_PCG_MAXITER;
            it = pb.pcg_max;
        }
    }
    pcg_iters += it;

    // ||Delta f_q||^2 = sum((dU^T dU) o H0), dU = x - U_q; then U_q <- x
    gram_lds<false>(n, r, 0, DiffF{x, Uq, n}, DiffF{x, Uq, n}, pb.S, r, nullptr, 0, s.scratch);
    for (int t = threadIdx.x; t < nr; t += WG) stg(Uq + t, ldg(x + t));
    __syncthreads();
    double part = 0.0;
    for (int t = threadIdx.x; t < r * r; t += WG) part = fma(pb.S[t], pb.H0[t], part);
    const double delta2 = wg_sum(part, s.red);
    refresh_dim(q, r0, lowp);
    return delta2;
}

// ------------------------------------------------------------------------------------
// balancing
// ------------------------------------------------------------------------------------

// Column norms from the panels themselves -> s.colnorm[k*r + l]
__device__ __forceinline__ void panel_colnorms() {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = pb.r;
    for (int kl = wave; kl < pb.d * r; kl += NWAVES) {
        const int k = kl / r, l = kl % r;
        const double* u = pb.U + pb.offU[k] + (int64_t)l * pb.n[k];
        double acc = 0.0;
        for (int i = lane; i < pb.n[k]; i += 64) acc = fma(u[i], u[i], acc);
        acc = wave_sum(acc);
        if (lane == 0) s.colnorm[kl] = sqrt(acc);
    }
    __syncthreads();
}

// Column norms from the Gram diagonals G_k[0,0][l,l].
__device__ __forceinline__ void gram_colnorms() {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r;
    for (int kl = threadIdx.x; kl < pb.d * r; kl += WG) {
        const int k = kl / r, l = kl % r;
        const int ld = pb.mA[k] * r;
        s.colnorm[kl] = sqrt(fmax(pb.G[pb.offG[k] + (int64_t)l * ld + l], 0.0));
    }
    __syncthreads();
}

// colnorm -> scale factors (in place); a column with a zero factor keeps scale 1.
__device__ __forceinline__ void balance_scales() {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r, d = pb.d;
    for (int l = threadIdx.x; l < r; l += WG) {
        bool zero = false;
        double lsum = 0.0;
        for (int k = 0; k < d; ++k) {
            const double nk = s.colnorm[k * r + l];
            if (!(nk > 0.0)) zero = true;
            else lsum += log(nk);
        }
        const double target = zero ? 0.0 : exp(lsum / d);
        for (int k = 0; k < d; ++k) {
            const double nk = s.colnorm[k * r + l];
            s.colnorm[k * r + l] = zero ? 1.0 : target / nk;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void scale_panels() {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r;
    for (int k = 0; k < pb.d; ++k) {
        const int n = pb.n[k];
        double* u = pb.U + pb.offU[k];
        for (int t = threadIdx.x; t < n * r; t += WG) u[t] *= s.colnorm[k * r + t / n];
    }
    __syncthreads();
}

// After a sweep: rescale panels and, consistently, the Grams and cross-Grams.
__device__ __forceinline__ void scale_grams(int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r;
    for (int k = 0; k < pb.d; ++k) {
        const int ld = pb.mA[k] * r;
        const double* sc = s.colnorm + k * r;
        double* G = pb.G + pb.offG[k];
        for (int t = threadIdx.x; t < ld * ld; t += WG) {
            const int i = t % ld, j = t / ld;
            G[t] *= sc[i % r] * sc[j % r];
        }
        double* X = pb.X + pb.offX[k];
        const int nx = ld * pb.mB[k] * r0;
        for (int t = threadIdx.x; t < nx; t += WG) X[t] *= sc[(t % ld) % r];
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------------
// the persistent kernel
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(WG) als_persistent(const Problem* __restrict__ problems, int count) {
    Smem& s = SMEM;
    const int pid = blockIdx.x;
    if (pid >= count) return;
    // problem descriptor -> LDS
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(problems + pid);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&s.pb);
        for (int t = threadIdx.x; t < (int)(sizeof(Problem) / 4); t += WG) dst[t] = src[t];
    }
    __syncthreads();
    const Problem& pb = s.pb;
    const int d = pb.d, r = pb.r;
    int64_t total_u = 0;
    for (int k = 0; k < d; ++k) total_u += (int64_t)pb.n[k] * r;

    for (int step = 0; step < pb.n_steps; ++step) {
        const int r0 = (step == 0) ? pb.r0 : r;
        if (step > 0) {
            // f_n <- previous result (same packed layout, rank r)
            for (int k = 0; k < d; ++k) {
                const int64_t cnt = (int64_t)pb.n[k] * r;
                for (int64_t t = threadIdx.x; t < cnt; t += WG) pb.V[pb.offV[k] + t] = pb.U[pb.offU[k] + t];
            }
            __syncthreads();
        }
        for (int k = 0; k < d; ++k) compute_Q(k, r0);
        panel_colnorms();
        balance_scales();
        scale_panels();
        // mixed-precision form: sweeps with FP32 contractions until the increment reaches the
        // FP32 floor (or the sweep budget is nearly spent), then one FP64 refinement sweep
        const bool mixed = pb.precision == CP_PREC_MIXED;
        bool lowp = mixed && pb.max_sweeps > 1;
        // (with tol = 0 the caller asks for exactly max_sweeps sweeps: FP32 until the last one)
        const double tol_low = pb.tol > 0.0 ? fmax(pb.tol, 1e-6) : 0.0;
        for (int k = 0; k < d; ++k) refresh_dim(k, r0, lowp);

        int sweeps = 0, pcg_iters = 0;
        uint32_t flags = CP_FLAG_NOT_CONVERGED;
        double eps = 0.0, fnorm = 0.0;
        for (int sw = 1; sw <= pb.max_sweeps; ++sw) {
            const bool was_low = lowp;
            double dmax2 = 0.0;
            for (int q = 0; q < d; ++q) {
                const double d2 = update_dim(q, r0, pcg_iters, flags, lowp);
                dmax2 = fmax(dmax2, d2);
            }
            // ||f||^2 = sum o_k U_k^T U_k
            double part = 0.0;
            for (int t = threadIdx.x; t < r * r; t += WG) {
                const int l = t % r, lp = t / r;
                double prod = 1.0;
                for (int k = 0; k < d; ++k) prod *= pb.G[pb.offG[k] + (int64_t)lp * (pb.mA[k] * r) + l];
                part += prod;
            }
            const double f2 = wg_sum(part, s.red);
            fnorm = sqrt(fmax(f2, 0.0));
            const double dmax = sqrt(fmax(dmax2, 0.0));
            eps = fnorm > 0.0 ? dmax / fnorm : dmax;
            gram_colnorms();
            balance_scales();
            scale_panels();
            scale_grams(r0);
            sweeps = sw;
            if (!isfinite(eps)) {
                flags |= CP_FLAG_NONFINITE;
                break;
            }
            if (was_low) {
                if (eps <= tol_low || sw + 1 >= pb.max_sweeps) {
                    // switch to FP64: recompute every Gram in FP64, then the refinement sweep
                    lowp = false;
                    for (int k = 0; k < d; ++k) refresh_dim(k, r0, false);
                }
                continue;
            }
            if (eps <= pb.tol) {
                flags &= ~CP_FLAG_NOT_CONVERGED;
                break;
            }
            if (mixed) break;   // the single FP64 refinement sweep is done
        }
        if (threadIdx.x == 0) {
            cp_als_report rep;
            rep.sweeps = sweeps;
            rep.pcg_iters = pcg_iters;
            rep.eps_conv = eps;
            rep.fnorm = fnorm;
            rep.flags = flags;
            rep.reserved = 0;
            pb.reports[step] = rep;
        }
        if (pb.traj) {
            double* dst = pb.traj + (int64_t)step * total_u;
            int64_t o = 0;
            for (int k = 0; k < d; ++k) {
                const int64_t cnt = (int64_t)pb.n[k] * r;
                for (int64_t t = threadIdx.x; t < cnt; t += WG) dst[o + t] = pb.U[pb.offU[k] + t];
                o += cnt;
            }
        }
        __syncthreads();
    }
}

size_t als_smem_bytes() { return sizeof(Smem); }

hipError_t launch_als(const Problem* d_problems, int count, hipStream_t stream) {
    const size_t smem = sizeof(Smem);
    hipError_t e = hipFuncSetAttribute((const void*)als_persistent, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(als_persistent, dim3(count), dim3(WG), smem, stream, d_problems, count);
    return hipGetLastError();
}

}  // namespace cpals
