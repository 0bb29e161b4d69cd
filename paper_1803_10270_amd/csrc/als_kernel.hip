// Persistent implicit CP-ALS kernel for gfx950: one workgroup, or a cluster of W workgroups
// that split the grid rows, advances one problem through n_steps implicit time steps,
// entirely on the device.
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
// preconditioner (H_q + lambda_q I) (x) I_n, H_q = o_{k != q} U_k^T U_k.
//
// Code layout: the kernel body is a small state machine (step set-up, Gram refresh,
// assembly, one composite product, increment, sweep end, report).  Every heavy routine is
// inlined at exactly one place, so the code a dimension update executes stays small
// (instruction-cache resident) and the register allocator sees one routine at a time.
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>
#include "dd_device.h"
#include "device_common.h"
#include "mfma_f64.h"

namespace cpals {

constexpr int XCDS = 8;          // XCDs of the device (MI355X), each with its own L2
constexpr int XCD_CUS = 32;      // compute units of one XCD
constexpr int TILE_PAR_N = 512;  // a cluster's Gram refresh forms whole tiles over grids up to this size
constexpr int SCRATCH = 16384;   // doubles of LDS shared by the phases of one dimension update
constexpr int LDS_PAIRS = 384;   // pair records of one dimension kept in LDS during assembly
constexpr int CG_TAPS = 5;       // stencils up to half bandwidth 2 keep their coefficients in registers

struct StageSlot {               // one staged Gram block of the assembly
    int64_t base;                // element offset of entry (0, 0) of the block
    int32_t ld;                  // its leading dimension, 0 for an empty slot
    int32_t pad;
};

extern __shared__ __attribute__((aligned(16))) unsigned char cpals_smem[];

struct Smem {
    Problem pb;
    OpDev ident;                 // the identity operator (preconditioner products)
    int32_t bnt[CP_MAX_OPS * CP_MAX_OPS];    // per operator block of the current product: taps
    int32_t boff[CP_MAX_OPS * CP_MAX_OPS];   // and first staged row of the stencil
    double red[2 * NWAVES];
    double dots[CP_MAX_OPS * CP_MAX_OPS * CP_MAX_RANK];
    double colnorm[CP_MAX_DIMS * CP_MAX_RANK];
    double gnrm[CP_MAX_DIMS];    // rank growth: t_k^T t_k
    double scratch[SCRATCH];
    PairRec pairs[LDS_PAIRS];
    StageSlot slots[(CP_MAX_DIMS - 1) * CP_MAX_OPS * CP_MAX_OPS];
    uint32_t iflag;
    int32_t part, W;             // this workgroup's index in the problem's cluster, cluster size
    uint32_t bar_target;         // arrivals the next cluster barrier waits for (thread 0)
    uint32_t sync_ok;            // 0 once a cluster barrier timed out
    uint32_t xlocal;             // 1: every workgroup of the cluster runs on this one XCD
    uint32_t dcount;             // calls of cluster_sum (selects the partial buffer)
    // operator blocks and coefficients of the matvec kept in LDS across the products of one
    // solve (key: the Kt array; cleared per solve)
    const double* kc_key;
    int32_t kc_base, kc_size, kc_rlo;
};
static_assert(sizeof(Smem) <= 160 * 1024, "LDS budget of one workgroup");

// The workgroup's LDS state, reached through the LDS symbol itself so that every access
// compiles to LDS instructions.
#define SMEM (*reinterpret_cast<Smem*>(cpals_smem))

// Workgroup-uniform copies (the values are equal in every lane; this tells the compiler).
__device__ __forceinline__ int ufirst(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double ufirst(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Row index i of a periodic grid of n points, for i a few periods off.
__device__ __forceinline__ int wrap_idx(int i, int n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

// ------------------------------------------------------------------------------------
// cluster of workgroups sharing one problem
// ------------------------------------------------------------------------------------

// Grid rows [rlo, rhi) of an n-row panel owned by this workgroup of the cluster.
__device__ __forceinline__ void own_rows(int n, int& rlo, int& rhi) {
    Smem& s = SMEM;
    const int W = ufirst(s.W), part = ufirst(s.part);
    const int per = n / W;
    rlo = part * per;
    rhi = rlo + per;
}

// Barrier of the cluster's workgroups (so that every write before it is visible to every
// workgroup after it).  The arrival counter only grows; a workgroup waits for W arrivals per
// barrier.  A wait is bounded: past the bound the barrier returns and sync_ok is cleared
// (the caller ends the problem).
// The wait ends with a device-scope acquire.  The arrival has two forms:
// - cluster spread over several XCDs: a device-scope release, which writes the dirty lines
//   of the XCD's L2 back to memory, since every XCD has an L2 of its own;
// - cluster on one XCD (xlocal): all members share one L2, which the vector L1s write
//   through, so it suffices that every wave's stores (and loads) have completed before the
//   arrival; the members' writes are not written back to memory at every barrier.
__device__ __forceinline__ void cluster_sync() {
    Smem& s = SMEM;
    const bool xl = ufirst((int)s.xlocal) != 0;
    if (xl) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (ufirst(s.W) == 1) return;
    if (tid_here() == 0) {
        const uint32_t tgt = s.bar_target + (uint32_t)s.W;
        s.bar_target = tgt;
        uint32_t* ctr = s.pb.bar;
        if (xl) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        long spins = 0;
        // spin on relaxed loads; one acquire fence once the count is reached (an acquire load
        // per spin would invalidate the L2 of the workgroup's XCD on every poll)
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tgt) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1l << 22)) {
                s.sync_ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// XCD of the executing wave (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ uint32_t xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u; }

// Whether the whole cluster runs on one XCD: every member sets its XCD's bit in a word of
// the barrier area (zeroed before the launch), a device-scope barrier publishes the bits,
// and every member reads the same mask.  Until then, and whenever the members are spread,
// the barriers keep the device-scope form.
__device__ __forceinline__ void detect_xcd_local() {
    Smem& s = SMEM;
    if (ufirst(s.W) == 1) return;
    uint32_t* mask = s.pb.bar + 16;
    if (tid_here() == 0) __hip_atomic_fetch_or(mask, 1u << xcd_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cluster_sync();
    if (tid_here() == 0) {
        const uint32_t m = __hip_atomic_load(mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s.xlocal = (m != 0u && (m & (m - 1u)) == 0u) ? 1u : 0u;
    }
    __syncthreads();
}

// sum_{w < W} base[w stride] in the order w = 0, 1, ...: the loads of up to 16 partials
// are in flight together (one round trip to memory for clusters of up to 16 workgroups)
__device__ __forceinline__ double sum_partials(const double* base, int64_t stride, int W) {
    constexpr int B = 16;
    double acc = 0.0;
    for (int w0 = 0; w0 < W; w0 += B) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = (w0 + u < W) ? ldg(base + (int64_t)(w0 + u) * stride) : 0.0;
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (w0 + u < W) acc += v[u];
    }
    return acc;
}

// E sums of that kind (base pointers b[e], nullptr for none) with all their loads in flight
// together, each in the order of sum_partials.
template <int E>
__device__ __forceinline__ void sum_partials_n(const double* const (&b)[E], int64_t stride, int W, double (&out)[E]) {
    constexpr int B = 16;
#pragma unroll
    for (int e = 0; e < E; ++e) out[e] = 0.0;
    for (int w0 = 0; w0 < W; w0 += B) {
        double v[E][B];
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int u = 0; u < B; ++u) v[e][u] = (w0 + u < W && b[e]) ? ldg(b[e] + (int64_t)(w0 + u) * stride) : 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (w0 + u < W) out[e] += v[e][u];
    }
}

// Sum over the cluster of one workgroup-uniform value, in a fixed order (partials in
// device memory, two alternating buffers so that a fast workgroup never overwrites a
// partial that a slow one has not read).
__device__ __forceinline__ double cluster_sum(double v) {
    Smem& s = SMEM;
    const int W = ufirst(s.W);
    if (W == 1) return v;
    const int part = ufirst(s.part);
    const int buf = ufirst((int)(s.dcount & 1u));
    double* base = s.pb.dpart + (int64_t)buf * W * 8;
    if (tid_here() == 0) stg(base + part * 8, v);
    cluster_sync();
    const double tot = sum_partials(base, 8, W);
    __syncthreads();
    if (tid_here() == 0) s.dcount += 1u;
    __syncthreads();
    return tot;
}

// Two workgroup-uniform values summed over the cluster behind one barrier (the second one
// carried from an earlier phase whose sum was not needed there); same order as cluster_sum.
__device__ __forceinline__ void cluster_sum2(double v, double u, double& sv, double& su) {
    Smem& s = SMEM;
    const int W = ufirst(s.W);
    if (W == 1) {
        sv = v;
        su = u;
        return;
    }
    const int part = ufirst(s.part);
    const int buf = ufirst((int)(s.dcount & 1u));
    double* base = s.pb.dpart + (int64_t)buf * W * 8;
    if (tid_here() == 0) {
        stg(base + part * 8, v);
        stg(base + part * 8 + 1, u);
    }
    cluster_sync();
    sv = sum_partials(base, 8, W);
    su = sum_partials(base + 1, 8, W);
    __syncthreads();
    if (tid_here() == 0) s.dcount += 1u;
    __syncthreads();
}

// Plain column-major panel element (i, c).
struct ColF {
    typedef double raw_t;
    const double* X;
    int ld;
    __device__ __forceinline__ static raw_t zero() { return 0.0; }
    __device__ __forceinline__ raw_t raw(int i, int c) const { return ldg(X + i + (int64_t)c * ld); }
    __device__ __forceinline__ double val(raw_t v) const { return v; }
};

// Rows rlo .. of a panel held in LDS, column c at X[c ld].
struct LdsColF {
    typedef double raw_t;
    const double* X;
    int rlo, ld;
    __device__ __forceinline__ static raw_t zero() { return 0.0; }
    __device__ __forceinline__ raw_t raw(int i, int c) const { return X[(i - rlo) + c * ld]; }
    __device__ __forceinline__ double val(raw_t v) const { return v; }
};

// x - u elementwise (the increment of one factor).
struct DiffF {
    typedef double2 raw_t;
    const double* x;
    const double* u;
    int ld;
    __device__ __forceinline__ static raw_t zero() { return double2{0.0, 0.0}; }
    __device__ __forceinline__ raw_t raw(int i, int c) const {
        const int64_t o = i + (int64_t)c * ld;
        return double2{ldg(x + o), ldg(u + o)};
    }
    __device__ __forceinline__ double val(raw_t v) const { return v.x - v.y; }
};

// Rows [rlo, rhi) of the stacked applied panel P = [O^0 X, O^1 X, ...] (n x m r, column
// a r + l) into `out`.
// For each batch of elements every tap and coefficient load is issued before the sums are
// formed.  Ends with a barrier.
// With ldo > 0, out is an LDS panel of the own rows: row i, column c at out[(i - rlo) + c ldo].
__device__ __forceinline__ void apply_panel(const OpDev* ops, int m, int n, int r, const double* X, double* out,
                                            int rlo, int rhi, int ldo = 0) {
    Smem& s = SMEM;
    for (int a = 0; a < m; ++a)
        if (ops[a].kind == CP_OP_RANK1) wg_coldots(n, r, ops[a].data + n, X, n, s.dots + a * r);
    const int nown = rhi - rlo;
    const int total = nown * m * r;
    const float invn = __frcp_rn((float)nown), invr = __frcp_rn((float)r);
    constexpr int U = 4;
    for (int t0 = tid_here(); t0 < total; t0 += U * WG) {
        double xv[U][CG_TAPS], cv[U][CG_TAPS];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
#pragma unroll
            for (int j = 0; j < CG_TAPS; ++j) xv[u][j] = cv[u][j] = 0.0;
            if (t < total) {
                const int c = fdiv(t, invn), i = rlo + (t - c * nown);
                const int a = fdiv(c, invr), l = c - a * r;
                const int kind = ops[a].kind, h = ops[a].hbw;
                const double* data = ops[a].data;
                const double* x = X + (int64_t)l * n;
                if (kind == CP_OP_IDENTITY) {
                    xv[u][0] = ldg(x + i);
                    cv[u][0] = 1.0;
                } else if (kind == CP_OP_DIAG) {
                    xv[u][0] = ldg(x + i);
                    cv[u][0] = ldg(data + i);
                } else if (kind == CP_OP_RANK1) {
                    xv[u][0] = s.dots[a * r + l];
                    cv[u][0] = ldg(data + i);
                } else if (h <= 2) {
#pragma unroll
                    for (int j = 0; j < CG_TAPS; ++j) {
                        if (j <= 2 * h) {
                            xv[u][j] = ldg(x + wrap_idx(i + j - h, n));
                            cv[u][j] = ldg(data + (int64_t)j * n + i);
                        }
                    }
                } else {
                    double v = 0.0;
                    for (int j = 0; j <= 2 * h; ++j) v = fma(ldg(data + (int64_t)j * n + i), ldg(x + wrap_idx(i + j - h, n)), v);
                    xv[u][0] = v;
                    cv[u][0] = 1.0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            if (t < total) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < CG_TAPS; ++j) v = fma(cv[u][j], xv[u][j], v);
                const int c = fdiv(t, invn), i = rlo + (t - c * nown);
                if (ldo) out[(i - rlo) + c * ldo] = v;
                else stg(out + i + (int64_t)c * n, v);
            }
        }
    }
    __syncthreads();
}

// Tiles t0 .. t1 - 1 of the Grams (the 16 x 16 tiles of G1 = P^T P on and above the
// diagonal in row-major triangular order, then those of G2 = P^T Q), each formed over all n
// rows of the published panels and stored (G1 also at its mirror).  The four waves split the
// rows (k-steps of four rows) and load their matrix-core operands straight from the panels,
// all loads of a batch in flight together; the partial tiles are added in LDS in wave order.
// Operands and result layout as in gram_lds.  Starts and ends with a barrier.
template <bool F32>
__device__ __forceinline__ void gram_tiles_direct(int n, int M1, int N2, const double* P, const double* Q, double* G1,
                                                  double* G2, int t0, int t1) {
    Smem& s = SMEM;
    constexpr int KB = 16;   // k-steps per batch of loads
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    const int kk = lane >> 4, cc = lane & 15;
    const int TM = (M1 + 15) >> 4;
    const int nt1 = TM * (TM + 1) / 2;
    const int S = (n + 3) >> 2;
    const int s0 = (wave * S) / NWAVES, s1 = ((wave + 1) * S) / NWAVES;
    double* red = s.scratch;   // [NWAVES - 1][4][64]
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        int ti, tj;
        const bool g1 = t < nt1;
        if (g1) {
            int a = 0, rem = t;
            while (rem >= TM - a) {
                rem -= TM - a;
                ++a;
            }
            ti = a;
            tj = a + rem;
        } else {
            ti = (t - nt1) % TM;
            tj = (t - nt1) / TM;
        }
        const int ca = ti * 16 + cc, cb = tj * 16 + cc;
        const bool oka = ca < M1, okb = cb < (g1 ? M1 : N2);
        const double* pa = P + (int64_t)(oka ? ca : 0) * n;
        const double* pbb = (g1 ? P : Q) + (int64_t)(okb ? cb : 0) * n;
        Tile<F32> acc;
        acc.zero();
        for (int sb = s0; sb < s1; sb += KB) {
            double av[KB], bv[KB];
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const int k = 4 * (sb + u) + kk;
                const bool ok = sb + u < s1 && k < n;
                av[u] = (ok && oka) ? ldg(pa + k) : 0.0;
                bv[u] = (ok && okb) ? ldg(pbb + k) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < KB; ++u) acc.step(bv[u], av[u]);
        }
        if (wave > 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) red[((wave - 1) * 4 + v) * 64 + lane] = acc.get(v);
        }
        __syncthreads();
        if (wave == 0) {
            for (int w = 1; w < NWAVES; ++w)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc.add(v, red[((w - 1) * 4 + v) * 64 + lane]);
            const int row = ti * 16 + cc;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = tj * 16 + Tile<F32>::row(lane, v);
                const double val = acc.get(v);
                if (g1) {
                    if (row < M1 && col < M1) {
                        stg(G1 + row + (int64_t)col * M1, val);
                        if (ti != tj) stg(G1 + col + (int64_t)row * M1, val);
                    }
                } else if (row < M1 && col < N2) {
                    stg(G2 + row + (int64_t)col * M1, val);
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// Gram refresh of one dimension: G_k = P_k^T P_k, X_k = P_k^T Q_k with P_k = [O^a U_k]_a
// (P_k formed once in the scratch panel, then both products over row chunks staged in LDS).
// U_k is read from `src` when given (a panel of the same layout that every workgroup has
// published, while U_k itself may still be written).  With `carry`, the workgroup-uniform
// cval is summed over the cluster behind the first barrier and the sum returned.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double refresh_dim(int k, int r0, bool lowp, const double* src = nullptr, bool carry = false,
                                              double cval = 0.0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[k], r = pb.r, m = pb.mA[k], mb = pb.mB[k];
    const double* Uk = src ? src : pb.U + pb.offU[k];
    int rlo, rhi;
    own_rows(n, rlo, rhi);
    const int M1 = m * r, N2 = mb * r0;
    const int W = ufirst(s.W);
    double* G1 = pb.G + pb.offG[k];
    double* G2 = pb.X + pb.offX[k];
    if (W > 1 && n <= TILE_PAR_N) {
        // a cluster on a short grid: the applied panel of the own rows is published, then
        // every workgroup forms whole tiles of G_q, X_q over all rows and stores them (the
        // barrier also sums a carried workgroup-uniform value); no partials, no reduction
        apply_panel(pb.opA[k], m, n, r, Uk, pb.P, rlo, rhi);
        const double csum = carry ? cluster_sum(cval) : (cluster_sync(), cval);
        const int TM = (M1 + 15) >> 4, TN = (N2 + 15) >> 4;
        const int ntiles = TM * (TM + 1) / 2 + TM * TN;
        const int part = ufirst(s.part);
        const int t0 = (part * ntiles) / W, t1 = ((part + 1) * ntiles) / W;
        if (lowp) gram_tiles_direct<true>(n, M1, N2, pb.P, pb.Q + pb.offQ[k], G1, G2, t0, t1);
        else gram_tiles_direct<false>(n, M1, N2, pb.P, pb.Q + pb.offQ[k], G1, G2, t0, t1);
        cluster_sync();
        return csum;
    }
    if (W > 1) {
        G1 = pb.gpart + (int64_t)ufirst(s.part) * pb.psz;
        G2 = G1 + M1 * M1;
    }
    ColF fb{pb.Q + pb.offQ[k], n};
    // a cluster's partials hold the tiles of G1 on and above the diagonal only; the
    // reduction below mirrors them
    const int nown = rhi - rlo;
    const int cap = SCRATCH - nown * M1;
    const int stage2 = 32 * ((((M1 + 15) >> 4) * 16 + 1) + (((N2 + 15) >> 4) * 16 + 1));   // two 16-row chunks
    if (!lowp && W > 1 && nown * M1 <= SCRATCH / 4 && stage2 <= cap) {
        // FP64 sweeps of a cluster: the applied panel of the own rows stays in LDS, above the
        // Gram routine's staging
        double* Pl = s.scratch + cap;
        apply_panel(pb.opA[k], m, n, r, Uk, Pl, rlo, rhi, nown);
        LdsColF fa{Pl, rlo, nown};
        gram_lds<false>(rlo, rhi, M1, N2, fa, fb, G1, M1, G2, M1, s.scratch, cap, false);
    } else {
        apply_panel(pb.opA[k], m, n, r, Uk, pb.P, rlo, rhi);
        ColF fa{pb.P, n};
        if (lowp) gram_lds<true>(rlo, rhi, M1, N2, fa, fb, G1, M1, G2, M1, s.scratch, SCRATCH, W == 1);
        else gram_lds<false>(rlo, rhi, M1, N2, fa, fb, G1, M1, G2, M1, s.scratch, SCRATCH, W == 1);
    }
    double csum = cval;
    if (W > 1) {
        // every workgroup adds up its slice of the entries over the cluster's partials (the
        // barrier also sums a carried workgroup-uniform value)
        if (carry) csum = cluster_sum(cval);
        else cluster_sync();
        // the work items: the 16 x 16 tiles of G1 on and above the diagonal (row tile <= column
        // tile, in the order of the Gram routine, 256 items each: 16 consecutive rows of a
        // column, then the next column), then the entries of G2; each G1 item is also stored
        // at its mirror
        const int TM = (M1 + 15) >> 4;
        const int nup = TM * (TM + 1) / 2 * 256;
        const int tot = nup + M1 * N2;
        const int per = (tot + W - 1) / W;
        const int e0 = ufirst(s.part) * per, e1 = min(tot, e0 + per);
        double* Gk = pb.G + pb.offG[k];
        double* Xk = pb.X + pb.offX[k];
        // offset of item e in a partial (and in G1 / after it for G2), -1 for tile padding
        auto at = [&](int e, int& i, int& j) {
            if (e >= nup) return M1 * M1 + (e - nup);
            int a = 0, rem = e >> 8;
            while (rem >= TM - a) {
                rem -= TM - a;
                ++a;
            }
            i = a * 16 + (e & 15);
            j = (a + rem) * 16 + ((e >> 4) & 15);
            return (i < M1 && j < M1) ? i + j * M1 : -1;
        };
        // three items per thread and pass, all their partials' loads in flight together
        for (int e = e0 + tid_here(); e < e1; e += 3 * WG) {
            const double* b[3];
            int off[3], ii[3], jj[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                ii[u] = jj[u] = 0;
                off[u] = e + u * WG < e1 ? at(e + u * WG, ii[u], jj[u]) : -1;
                b[u] = off[u] >= 0 ? pb.gpart + off[u] : nullptr;
            }
            double a[3];
            sum_partials_n<3>(b, pb.psz, W, a);
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                if (!b[u]) continue;
                if (off[u] >= M1 * M1) {
                    stg(Xk + (off[u] - M1 * M1), a[u]);
                } else {
                    stg(Gk + off[u], a[u]);
                    if ((ii[u] >> 4) != (jj[u] >> 4)) stg(Gk + jj[u] + (int64_t)ii[u] * M1, a[u]);
                }
            }
        }
        cluster_sync();
    }
    return csum;
}

// Q_k = [O_B^b V_k]_b for every dimension (the fixed B-side panels of a time step).
__device__ __forceinline__ void compute_Q_all(int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    for (int k = 0; k < pb.d; ++k) {
        const int n = pb.n[k], mb = pb.mB[k];
        const double* Vk = pb.V + pb.offV[k];
        for (int b = 0; b < mb; ++b)
            if (pb.opB[k][b].kind == CP_OP_RANK1) wg_coldots(n, r0, pb.opB[k][b].data + n, Vk, n, s.dots + b * r0);
        for (int b = 0; b < mb; ++b) apply_op(pb.opB[k][b], n, r0, Vk, n, pb.Q + pb.offQ[k] + (int64_t)b * r0 * n, n, s.dots + b * r0);
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// Hadamard assembly (eqs. ML, MR): one pass over the r x rc position grid of dimension q,
//   out[l + (blk rc + lc) r] = sum over the pair records of block blk of
//                              coef * prod_{j-th dim k != q} src_k[block slot_j][l, lc]
// (src = G for the C blocks, X for the D blocks).  Per chunk of E = 64 PG positions the
// entries of every (dimension, operator block) slot are staged in LDS; wave w takes the 64
// positions of group w % PG and the share w / PG of every block's pair list, so that all
// lanes of a wave walk the same pair records (uniform slot branches; slot 0 is held in
// registers).  The shares meet in LDS and are added in a fixed order.  With H0 also
// H0 = prod_j src_k[slot 0] and the trace sum_blk trace(C^blk) <O^a, O^b>_F are produced.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double hadamard_pass(int q, bool withH0, int rc, int MM, const double* src, int nblk,
                                                const int32_t* off, const PairRec* pairs_g, double* out,
                                                const double* trOO) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d, r = pb.r;
    const int nk = ufirst(d - 1);
    const int nE = r * rc;
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    const int p0 = off[0], np = off[nblk] - off[0];
    __syncthreads();
    const bool pl = np <= LDS_PAIRS;
    if (pl) {
        for (int t = tid_here(); t < np; t += WG) {
            const double* src_rec = reinterpret_cast<const double*>(pairs_g + p0 + t);
            double* dst_rec = reinterpret_cast<double*>(s.pairs + t);
            dst_rec[0] = ldg(src_rec);
            dst_rec[1] = ldg(src_rec + 1);
        }
    }
    for (int t = tid_here(); t < nk * MM; t += WG) {
        const int j = t / MM, ab = t % MM;
        const int k = j < q ? j : j + 1;
        const int mk = pb.mA[k];
        const int nb = withH0 ? mk : pb.mB[k];
        StageSlot sl;
        sl.pad = 0;
        if (ab < mk * nb) {
            const int a = ab % mk, b = ab / mk;
            sl.ld = mk * r;
            sl.base = (withH0 ? pb.offG[k] : pb.offX[k]) + (int64_t)(b * rc) * sl.ld + a * r;
        } else {
            sl.ld = 0;
            sl.base = 0;
        }
        s.slots[t] = sl;
    }
    // chunk geometry: PG groups of 64 positions, SPL = NWAVES / PG shares of the pair lists
    const int W = ufirst(s.W), cpart = ufirst(s.part);
    int PG = NWAVES;
    while (PG > 1 && (64 * PG * (nk * MM + (NWAVES / PG) * nblk) > SCRATCH || (nE + 64 * PG - 1) / (64 * PG) < W))
        PG >>= 1;
    PG = ufirst(PG);
    const int SPL = NWAVES / PG;
    const int E = 64 * PG;
    const int pg = wave % PG, sp = wave / PG;
    const int e = pg * 64 + lane;
    double* st = s.scratch;
    double* part = st + nk * MM * E;
    const float invr = __frcp_rn((float)r);
    __syncthreads();
    double trpart = 0.0;
    for (int e0 = cpart * E; e0 < nE; e0 += W * E) {
        // stage the slot entries of positions e0 .. e0 + E (a thread keeps one position)
        {
            const int ee = tid_here() & (E - 1);
            const int spos = e0 + ee;
            const int slc = fdiv(spos, invr), sl0 = spos - slc * r;
            const bool ok = spos < nE;
            const int nslot = nk * MM, step = WG / E;
            for (int sb = tid_here() / E; sb < nslot; sb += 16 * step) {
                double v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int sl = sb + u * step;
                    v[u] = 0.0;
                    if (sl < nslot) {
                        const StageSlot ss = s.slots[sl];
                        if (ok && ss.ld) v[u] = ldg(src + ss.base + (int64_t)slc * ss.ld + sl0);
                    }
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int sl = sb + u * step;
                    if (sl < nslot) st[sl * E + ee] = v[u];
                }
            }
        }
        __syncthreads();
        const int pos = e0 + e;
        double h0r[CP_MAX_DIMS - 1];
#pragma unroll
        for (int j = 0; j < CP_MAX_DIMS - 1; ++j) h0r[j] = (j < nk) ? st[(j * MM) * E + e] : 1.0;
        if (withH0 && sp == 0 && pos < nE) {
            double prod = 1.0;
#pragma unroll
            for (int j = 0; j < CP_MAX_DIMS - 1; ++j) prod *= h0r[j];
            stg(pb.H0 + pos, prod);
        }
        // pair products, instantiated per number of factors so that every factor read is
        // unconditional: four records at a time, all their LDS reads in flight together
        auto pairs_fast = [&](auto nk_c) {
            constexpr int NK = decltype(nk_c)::value;
            for (int blk = 0; blk < nblk; ++blk) {
                const int b0 = off[blk] - p0, len = off[blk + 1] - off[blk];
                const int lo = ufirst(b0 + (len * sp) / SPL), hi = ufirst(b0 + (len * (sp + 1)) / SPL);
                double acc4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int pi = lo; pi < hi; pi += 4) {
                    double coef[4];
                    uint64_t sw[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const bool ok = pi + u < hi;
                        const int pp = ok ? pi + u : lo;
                        coef[u] = ok ? s.pairs[pp].coef : 0.0;
                        sw[u] = *reinterpret_cast<const uint64_t*>(s.pairs[pp].slot);
                    }
                    double f[4][NK > 0 ? NK : 1];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int j = 0; j < NK; ++j) f[u][j] = st[(j * MM + (int)((sw[u] >> (8 * j)) & 0xffu)) * E + e];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        double prod = coef[u];
#pragma unroll
                        for (int j = 0; j < NK; ++j) prod *= f[u][j];
                        acc4[u] += prod;
                    }
                }
                part[(sp * nblk + blk) * E + e] = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
            }
        };
        if (pl) {
            switch (nk) {
                case 1: pairs_fast(std::integral_constant<int, 1>{}); break;
                case 2: pairs_fast(std::integral_constant<int, 2>{}); break;
                case 3: pairs_fast(std::integral_constant<int, 3>{}); break;
                case 4: pairs_fast(std::integral_constant<int, 4>{}); break;
                case 5: pairs_fast(std::integral_constant<int, 5>{}); break;
                case 6: pairs_fast(std::integral_constant<int, 6>{}); break;
                default: pairs_fast(std::integral_constant<int, 7>{}); break;
            }
        } else {
            // pair list too long for LDS: records from device memory, one at a time
            for (int blk = 0; blk < nblk; ++blk) {
                const int b0 = off[blk] - p0, len = off[blk + 1] - off[blk];
                const int lo = ufirst(b0 + (len * sp) / SPL), hi = ufirst(b0 + (len * (sp + 1)) / SPL);
                double acc = 0.0;
                for (int pi = lo; pi < hi; ++pi) {
                    const double* rec = reinterpret_cast<const double*>(pairs_g + p0 + pi);
                    const double coef = ldg(rec);
                    const uint64_t sw = (uint64_t)__double_as_longlong(ldg(rec + 1));
                    double prod = coef;
                    for (int j = 0; j < nk; ++j) prod *= st[(j * MM + (int)((sw >> (8 * j)) & 0xffu)) * E + e];
                    acc += prod;
                }
                part[(sp * nblk + blk) * E + e] = acc;
            }
        }
        __syncthreads();
        for (int t = tid_here(); t < nblk * E; t += WG) {
            const int blk = t / E, ee = t & (E - 1);
            const int p = e0 + ee;
            if (p < nE) {
                double acc = 0.0;
                for (int u = 0; u < SPL; ++u) acc += part[(u * nblk + blk) * E + ee];
                const int lc = fdiv(p, invr), l = p - lc * r;
                stg(out + l + (int64_t)(blk * rc + lc) * r, acc);
                if (withH0 && l == lc) trpart = fma(acc, trOO[blk], trpart);
            }
        }
        __syncthreads();
    }
    return trpart;
}

// C, D and H0 of dimension q; returns trace(M_q) (without the shift).
__device__ __forceinline__ double assemble(int q, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d, r = pb.r, mq = pb.mA[q], mbq = pb.mB[q];
    double trpart = 0.0;
    if (d == 1) {
        // every Hadamard product over k != q is empty (all ones)
        for (int t = tid_here(); t < mq * mq * r * r; t += WG) {
            const int blk = t / (r * r), e = t % (r * r);
            const int l = e % r, lp = e / r;
            double acc = 0.0;
            for (int pi = pb.offC[q][blk]; pi < pb.offC[q][blk + 1]; ++pi) acc += ldg(&pb.pairsC[pi].coef);
            stg(pb.Cm + l + (int64_t)(blk * r + lp) * r, acc);
            if (l == lp) trpart = fma(acc, pb.trOO[q][blk], trpart);
        }
        for (int t = tid_here(); t < mq * mbq * r * r0; t += WG) {
            const int blk = t / (r * r0), e = t % (r * r0);
            const int l = e % r, l0 = e / r;
            double acc = 0.0;
            for (int pi = pb.offD[q][blk]; pi < pb.offD[q][blk + 1]; ++pi) acc += ldg(&pb.pairsD[pi].coef);
            stg(pb.Dm + l + (int64_t)(blk * r0 + l0) * r, acc);
        }
        for (int t = tid_here(); t < r * r; t += WG) stg(pb.H0 + t, 1.0);
        return wg_sum(trpart, s.red);
    }
    for (int pass = 0; pass < 2; ++pass) {
        const bool c = pass == 0;
        trpart += hadamard_pass(q, c, c ? r : r0, c ? pb.MMq[q] : pb.MXq[q], c ? pb.G : pb.X, c ? mq * mq : mq * mbq,
                                c ? pb.offC[q] : pb.offD[q], c ? pb.pairsC : pb.pairsD, c ? pb.Cm : pb.Dm, pb.trOO[q]);
    }
    // (the cluster sum's barrier publishes the C, D and H0 entries of every workgroup)
    return cluster_sum(wg_sum(trpart, s.red));
}

// ------------------------------------------------------------------------------------
// Preconditioner: Hinv = (H0 + lam I)^{-1} by Gauss-Jordan elimination on the diagonal
// pivots (H0 + lam I is symmetric positive definite).  The matrix lives in LDS in two
// buffers; for pivot p every thread reads its entries, the pivot row and column from one
// buffer and writes its updated entries to the other, so each pivot costs one barrier and
// no thread branches on its position.  1 / pivot is the hardware reciprocal refined by two
// Newton steps (within an ulp of the quotient).  Returns flags.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double recip_nr(double a) {
    double x = __builtin_amdgcn_rcp(a);
    x = fma(x, fma(-a, x, 1.0), x);
    x = fma(x, fma(-a, x, 1.0), x);
    return x;
}

template <int PER>
__device__ __forceinline__ uint32_t factor_precond_t(double lam) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r, rr = r * r;
    double* M0 = s.scratch;               // [2][r r], column-major: entry (i, j) at i + j r
    double* M1 = s.scratch + rr;
    const float invr = __frcp_rn((float)r);
    // entry u of this thread: t = tid + u WG = i + j r; entries past r r read entry 0 and are
    // never written
    int hi[PER], hj[PER];
    double dmax = 0.0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = tid_here() + u * WG;
        const int j = fdiv(t, invr);
        hi[u] = (t < rr) ? t - j * r : 0;
        hj[u] = (t < rr) ? j : 0;
        if (t < rr) {
            double v = ldg(pb.H0 + t);
            if (hi[u] == hj[u]) {
                v += lam;
                dmax = fmax(dmax, v);
            }
            M0[t] = v;
        }
    }
    dmax = wave_max(dmax);
    if ((tid_here() & 63) == 0) s.red[tid_here() >> 6] = dmax;
    __syncthreads();
    dmax = 0.0;
    for (int w = 0; w < NWAVES; ++w) dmax = fmax(dmax, s.red[w]);
    uint32_t fl = 0;
    // In-place Gauss-Jordan step on pivot p, with selects in place of branches:
    //   row p: h[p][j] / piv (1 / piv on the diagonal); column p: -h[i][p] / piv;
    //   elsewhere h[i][j] - h[i][p] h[p][j] / piv.
    auto pivot = [&](int p, const double* Mc, double* Mn) __attribute__((always_inline)) {
        double piv = Mc[p + p * r];
        if (!(piv > 1e-12 * dmax)) fl |= CP_FLAG_REGULARIZED;
        if (!(piv > 0.0)) piv = (lam > 0.0) ? lam : 1e-300;
        double hv[PER], cv[PER], rv[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            hv[u] = Mc[hi[u] + hj[u] * r];
            cv[u] = Mc[hi[u] + p * r];
            rv[u] = Mc[p + hj[u] * r];
        }
        const double ip = recip_nr(piv);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = hi[u], j = hj[u];
            const double e = (j == p) ? 1.0 : rv[u];
            const double base = (j == p) ? 0.0 : hv[u];
            const double nv = (i == p) ? e * ip : fma(-cv[u] * ip, e, base);
            if (tid_here() + u * WG < rr) Mn[i + j * r] = nv;
        }
        __syncthreads();
    };
    for (int p = 0; p < r; p += 2) {
        pivot(p, M0, M1);
        if (p + 1 < r) pivot(p + 1, M1, M0);
    }
    // the result is in M0 when r is even, else in M1; symmetrised (the preconditioner of CG
    // must be symmetric)
    const double* Mr = (r & 1) ? M1 : M0;
    double* Hout = pb.Hinv + (int64_t)ufirst(s.part) * rr;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = tid_here() + u * WG;
        if (t < rr) stg(Hout + t, 0.5 * (Mr[t] + Mr[hj[u] + hi[u] * r]));
    }
    __syncthreads();
    return fl;
}

// The value of lane `src` (a compile-time constant after unrolling) in every lane.
__device__ __forceinline__ double readlane_f64(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// r <= 32: wave 0 alone inverts the 32 x 32 matrix [H0 + lam I, 0; 0, I] by Gauss-Jordan in
// registers.  The matrix is an 8 x 8 grid of 4 x 4 blocks, lane l holding block
// (l >> 3, l & 7); for pivot p the pivot, the four pivot-row entries of the lane's columns
// and the four pivot-column entries of the lane's rows arrive by cross-lane permutes (nine
// per pivot), so the 32 pivots need no workgroup barrier.  The pivot loop is unrolled so that
// every register index is fixed.  Same arithmetic per entry as the LDS form above
// (select-based update, Newton-refined reciprocal); the padding block stays the identity and
// does not touch the leading r x r block.
__device__ __forceinline__ uint32_t factor_precond_wave(double lam) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r, rr = r * r;
    __syncthreads();
    if (tid_here() < 64) {
        const int lane = tid_here();
        const int bi = lane >> 3, bj = lane & 7;
        double M[4][4];
        double dmax = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = 4 * bi + a, j = 4 * bj + b;
                double v = (i == j) ? 1.0 : 0.0;
                if (i < r && j < r) v = ldg(pb.H0 + i + j * r);
                M[a][b] = v;
            }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = 4 * bi + a, j = 4 * bj + b;
                if (i == j && i < r) {
                    M[a][b] += lam;
                    dmax = fmax(dmax, M[a][b]);
                }
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        uint32_t fl = 0;
#pragma unroll
        for (int p = 0; p < 32; ++p) {
            const int bp = p >> 2, pa = p & 3;
            // the pivot from its fixed lane by scalar reads (no LDS round trip on the chain)
            double piv = readlane_f64(M[pa][pa], 9 * bp);
            if (p < r) {
                if (!(piv > 1e-12 * dmax)) fl |= CP_FLAG_REGULARIZED;
                if (!(piv > 0.0)) piv = (lam > 0.0) ? lam : 1e-300;
            }
            const double ip = recip_nr(piv);
            double rv[4], cv[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) rv[b] = __shfl(M[pa][b], 8 * bp + bj, 64);   // A[p][4 bj + b]
#pragma unroll
            for (int a = 0; a < 4; ++a) cv[a] = __shfl(M[a][pa], 8 * bi + bp, 64);   // A[4 bi + a][p]
            // entry (i, j) = (4 bi + a, 4 bj + b) lies in the pivot row only if a == pa and
            // bi == bp, in the pivot column only if b == pa and bj == bp: the register index
            // settles the first half of each test at compile time
            const bool prow = bi == bp, pcol = bj == bp;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double mc = -cv[a] * ip;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const bool jp = (b == pa) && pcol;
                    const double e = jp ? 1.0 : rv[b];
                    const double base = jp ? 0.0 : M[a][b];
                    const double upd = fma(mc, e, base);
                    M[a][b] = ((a == pa) && prow) ? e * ip : upd;
                }
            }
        }
        // symmetrised (the preconditioner of CG must be symmetric) through a copy in LDS
        double* T = s.scratch;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) T[(4 * bi + a) + 32 * (4 * bj + b)] = M[a][b];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double* Hout = pb.Hinv + (int64_t)ufirst(s.part) * rr;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = 4 * bi + a, j = 4 * bj + b;
                if (i < r && j < r) stg(Hout + i + j * r, 0.5 * (M[a][b] + T[j + 32 * i]));
            }
        if (lane == 0) s.iflag = fl;
    }
    __syncthreads();
    return s.iflag;
}

__device__ __forceinline__ uint32_t factor_precond(double lam) {
    constexpr int PER_FULL = (CP_MAX_RANK * CP_MAX_RANK + WG - 1) / WG;
    return (SMEM.pb.r <= 32) ? factor_precond_wave(lam) : factor_precond_t<PER_FULL>(lam);
}

// ------------------------------------------------------------------------------------
// Composite product on the matrix cores:
//   out[i, j] = sum_blk sum_{l < rc} (comp_blk X)[i, l] Kt[j + (blk rc + l) r]   (i < n, j < r)
// then, with `shift`, out += lam X and, with `dot`, the return value sum_ij X[i, j] out[i, j]
// (per thread; both need rc == r).  Used for the right-hand side (comp = (O_A^a)^T O_B^b, Kt = D blocks)
// and the matvec (M_q + lam I) p (comp = (O^a)^T O^b, Kt = C blocks); the preconditioner has a
// row-local routine of its own (precond_apply).
//
// X is staged in LDS pass by pass (up to 16 SPW NWAVES rows plus a halo of the widest
// stencil); each lane forms the A fragment it feeds to the matrix core directly from the
// staged rows and its stencil coefficients (held in registers), so the stacked panel
// [comp_blk X] is never stored.  The r x rc block of Kt of the next operator block is
// prefetched into registers while the current one is consumed from LDS.
//
// The panel is produced by the transform xf while it is staged (v = a + beta b, written back
// to wv, and x2 += alpha2 p2 on the same elements): the conjugate-gradient vector updates
// ride along with the product that consumes their result.
// ------------------------------------------------------------------------------------
struct Xform {
    const double* a;
    const double* b;     // optional
    double beta;
    double* wv;          // optional: v is written here
    double* x2;          // optional: x2 += alpha2 * p2
    const double* p2;
    double alpha2;
    double* acopy;       // optional (modes 2 and 3): a itself is written here
};

// Transform of the rows [rlo, rlo + nown) of an n-row panel of rc columns (ld n): all loads
// of a batch are issued before any store.  MODE 0: v = a; 1: v = a, wv = v; 2: v = a + beta b,
// wv = v (and acopy = a when given); 3: as 2 and x2 += alpha2 p2.  With `lds`, v goes to
// Xs[l ldx + H + (i - rlo)] and, given Xa, the untransformed a to the same place of Xa.
template <int MODE>
__device__ __forceinline__ void xform_rows(const Xform& xf, int n, int rlo, int nown, int rc, bool lds, double* Xs,
                                           int ldx, int H, double* Xa) {
    constexpr int U = 4;
    const int total = nown * rc;
    const float invn = __frcp_rn((float)nown);
    for (int t0 = tid_here(); t0 < total; t0 += U * WG) {
        double va[U], vb[U], vx[U], vp[U];
        int64_t idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            const bool ok = t < total;
            const int l = fdiv(t, invn);
            idx[u] = (int64_t)(rlo + (t - l * nown)) + (int64_t)l * n;
            va[u] = ok ? ldg(xf.a + idx[u]) : 0.0;
            vb[u] = (MODE >= 2 && ok) ? ldg(xf.b + idx[u]) : 0.0;
            vx[u] = (MODE == 3 && ok) ? ldg(xf.x2 + idx[u]) : 0.0;
            vp[u] = (MODE == 3 && ok) ? ldg(xf.p2 + idx[u]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            if (t < total) {
                const double v = (MODE >= 2) ? fma(xf.beta, vb[u], va[u]) : va[u];
                if (MODE >= 1) stg(xf.wv + idx[u], v);
                if (MODE >= 2 && xf.acopy) stg(xf.acopy + idx[u], va[u]);
                if (MODE == 3) stg(xf.x2 + idx[u], fma(xf.alpha2, vp[u], vx[u]));
                if (lds) {
                    const int l = fdiv(t, invn);
                    Xs[l * ldx + H + (t - l * nown)] = v;
                    if (Xa) Xa[l * ldx + H + (t - l * nown)] = va[u];
                }
            }
        }
    }
}

__device__ __forceinline__ void xform_dispatch(const Xform& xf, int n, int rlo, int nown, int rc, bool lds, double* Xs,
                                               int ldx, int H, double* Xa = nullptr) {
    const int mode = xf.x2 ? 3 : (xf.b ? 2 : (xf.wv ? 1 : 0));
    switch (ufirst(mode)) {
        case 0: xform_rows<0>(xf, n, rlo, nown, rc, lds, Xs, ldx, H, Xa); break;
        case 1: xform_rows<1>(xf, n, rlo, nown, rc, lds, Xs, ldx, H, Xa); break;
        case 2: xform_rows<2>(xf, n, rlo, nown, rc, lds, Xs, ldx, H, Xa); break;
        default: xform_rows<3>(xf, n, rlo, nown, rc, lds, Xs, ldx, H, Xa); break;
    }
}


// Staging of one pass with the transform fused: rows i0 - H .. i0 + nrow + H (periodic) of
// v (MODE as in xform_rows) go to Xs[l ldx + j]; the pass rows (H <= j < H + nrow) also
// write wv (and, MODE 3, x2 += alpha2 p2).  Halo rows are formed from the transform's
// inputs, which the caller guarantees are not rewritten by this transform.
template <int MODE>
__device__ __forceinline__ void xform_stage(const Xform& xf, int n, int i0, int nrow, int H, int rc, double* Xs,
                                            int ldx) {
    constexpr int U = 4;
    const int R = nrow + 2 * H;
    const int total = R * rc;
    const float invR = __frcp_rn((float)R);
    for (int t0 = tid_here(); t0 < total; t0 += U * WG) {
        double va[U], vb[U], vx[U], vp[U];
        int64_t idx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            const bool ok = t < total;
            const int l = fdiv(t, invR), j = t - l * R;
            const bool own = ok && j >= H && j < H + nrow;
            idx[u] = (int64_t)wrap_idx(i0 - H + j, n) + (int64_t)l * n;
            va[u] = ok ? ldg(xf.a + idx[u]) : 0.0;
            vb[u] = (MODE >= 2 && ok) ? ldg(xf.b + idx[u]) : 0.0;
            vx[u] = (MODE == 3 && own) ? ldg(xf.x2 + idx[u]) : 0.0;
            vp[u] = (MODE == 3 && own) ? ldg(xf.p2 + idx[u]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * WG;
            if (t < total) {
                const int l = fdiv(t, invR), j = t - l * R;
                const bool own = j >= H && j < H + nrow;
                const double v = (MODE >= 2) ? fma(xf.beta, vb[u], va[u]) : va[u];
                Xs[l * ldx + j] = v;
                if (MODE >= 1 && own) stg(xf.wv + idx[u], v);
                if (MODE == 3 && own) stg(xf.x2 + idx[u], fma(xf.alpha2, vp[u], vx[u]));
            }
        }
    }
}

__device__ __forceinline__ void xform_stage_dispatch(const Xform& xf, int n, int i0, int nrow, int H, int rc, double* Xs,
                                                     int ldx) {
    const int mode = xf.x2 ? 3 : (xf.b ? 2 : (xf.wv ? 1 : 0));
    switch (ufirst(mode)) {
        case 0: xform_stage<0>(xf, n, i0, nrow, H, rc, Xs, ldx); break;
        case 1: xform_stage<1>(xf, n, i0, nrow, H, rc, Xs, ldx); break;
        case 2: xform_stage<2>(xf, n, i0, nrow, H, rc, Xs, ldx); break;
        default: xform_stage<3>(xf, n, i0, nrow, H, rc, Xs, ldx); break;
    }
}

template <bool F32, int TN>
__device__ __forceinline__ double cgemm(int n, int r, const OpDev* comps, int nblk, int rc, Xform xf,
                                        const double* Kt, double* out, double lam, bool shift, bool dot, int rlo, int rhi,
                                        bool keepable) {
    constexpr int SPW = (TN == 4) ? 2 : 4;   // 16-row strips per wave and pass
    constexpr int LDB = TN * 16 + 1;
    constexpr int PF = (64 * TN * 16 + WG - 1) / WG;
    Smem& s = SMEM;
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    const int rc4 = (rc + 3) & ~3;
    const int ktsz = rc4 * LDB;
    // the operator blocks' shapes, one block per lane (nblk <= 16), reduced over the wave:
    // H the widest half-bandwidth, rank-1 blocks, and whether every block is an identity,
    // diagonal or band of at most 5 taps (the flat k-step split) with its widest tap count
    int bk = CP_OP_IDENTITY, bh = 0;
    if (lane < nblk) {
        bk = comps[lane].kind;
        bh = comps[lane].hbw;
    }
    const bool bband = bk == CP_OP_BAND;
    const int H = ufirst((int)wave_max((double)(bband ? bh : 0)));
    const bool any_r1 = __ballot(bk == CP_OP_RANK1) != 0;
    const bool flat_ok = !any_r1 && __ballot(bband && bh > 2) == 0;
    const int flat_taps = ufirst((int)wave_max((double)(bband ? 2 * bh + 1 : 1)));
    if (tid_here() < nblk) {
        s.bnt[tid_here()] = bband ? 2 * bh + 1 : 1;
        s.boff[tid_here()] = bband ? H - bh : H;
    }
    // rows per pass: as many strips as the waves hold, limited by the LDS staging area
    const int nown = rhi - rlo;
    int RP = min((nown + 15) >> 4, NWAVES * SPW) * 16;
    auto ldx_of = [&](int rp) { return ((rp + 2 * H + 15) & ~31) + 16; };   // odd multiple of 16
    while (RP > 16 && ldx_of(RP) * rc + 2 * ktsz + 2 * CG_TAPS * RP > SCRATCH) RP -= 16;
    RP = ufirst(RP);
    const int ldx = ldx_of(RP);
    const int R = RP + 2 * H;
    const int npass = (nown + RP - 1) / RP;
    // one pass over the whole grid: the halo is copied from the staged rows; otherwise own
    // rows come from the transformed panel and halo rows are formed from the transform's
    // inputs (never rewritten in place when there is a halo: p is double-buffered)
    const bool single = nown == n && npass == 1;
    // When every operator block's Kt rows and stencil coefficients fit in LDS beside the
    // staged rows (short passes: a cluster's share of the grid), they are staged once per
    // pass; otherwise block b + 1 is prefetched while block b is consumed.
    const bool allk = ufirst((int)(ldx * rc + nblk * (ktsz + CG_TAPS * RP) <= SCRATCH)) != 0;
    // Kept blocks (one pass, every block staged): they sit at the top of the scratch area, the
    // staged rows and the reduction area of the block split at the bottom.  They are reused
    // when key, place and rows match.
    const int REDSZ = NWAVES * TN * 256;
    const int SA = nblk * (ktsz + CG_TAPS * RP);
    const int kbase = SCRATCH - SA;
    const bool keep = ufirst((int)(keepable && allk && npass == 1 && ldx * rc + REDSZ <= kbase)) != 0;
    const bool hit = keep && ufirst((int)(s.kc_key == Kt && s.kc_base == kbase && s.kc_size == SA &&
                                          s.kc_rlo == rlo)) != 0;
    double* Xs = s.scratch;
    double* KtS = keep ? s.scratch + kbase : s.scratch + ldx * rc;   // [nkb][rc4][LDB]
    double* CfS = KtS + (allk ? nblk : 2) * ktsz;        // [nkb][CG_TAPS][RP] stencil coefficients
    const bool xw = xf.wv != nullptr || xf.x2 != nullptr;
    const double* own_src = xw ? xf.wv : xf.a;
    // the transform rides along with the staging of each pass unless the rank-1 blocks need
    // the whole transformed panel first, or a halo row could be read after being rewritten
    const bool fused = !single && !any_r1 &&
                       (H == 0 || (xf.wv != xf.a && xf.wv != xf.b && xf.x2 != xf.a && xf.x2 != xf.b));
    __syncthreads();
    if (xw && !single && !fused) {
        // apply the transform to the own rows first
        xform_dispatch(xf, n, rlo, nown, rc, false, nullptr, 0, 0);
        __syncthreads();
    }
    if (any_r1 && !single) {
        // rank-1 blocks: dots[blk rc + l] = w_blk^T X[:, l] from the full panel
        for (int b = 0; b < nblk; ++b) {
            if (comps[b].kind != CP_OP_RANK1) continue;
            const double* w = comps[b].data + n;
            for (int l = wave; l < rc; l += NWAVES) {
                double acc = 0.0;
                for (int i = lane; i < n; i += 64) acc = fma(ldg(w + i), ldg(own_src + i + (int64_t)l * n), acc);
                acc = wave_sum(acc);
                if (lane == 0) s.dots[b * rc + l] = acc;
            }
        }
    }
    double part = 0.0;
    for (int i0 = rlo; i0 < rhi; i0 += RP) {
        const int tid = tid_here();
        const int lane = tid & 63, wave = tid >> 6;
        const int kq = lane >> 4, cc = lane & 15;
        const int nrow = min(RP, rhi - i0);
        const int nsp = (nrow + 15) >> 4;
        // fewer strips than waves with every block staged: the waves split the operator
        // blocks (G groups per strip) and their partial tiles are added afterwards
        const int G = (allk && nsp < NWAVES && NWAVES % nsp == 0 &&
                       NWAVES * TN * 256 <= (keep ? REDSZ : SCRATCH - ldx * rc)) ? NWAVES / nsp : 1;
        const int kg = G > 1 ? wave / nsp : 0;
        const int wstrip = G > 1 ? wave - kg * nsp : wave;
        // stage X rows i0 - H .. i0 + RP + H (periodic); in a single pass the halo is copied
        // from the staged rows afterwards (they may be rewritten by the transform)
        if (single) {
            xform_dispatch(xf, n, 0, n, rc, true, Xs, ldx, H);
        } else if (fused) {
            xform_stage_dispatch(xf, n, i0, nrow, H, rc, Xs, ldx);
        } else {
            const float invR = __frcp_rn((float)R);
            batched_loop<4>(
                R * rc,
                [&](int t) {
                    const int l = fdiv(t, invR);
                    const int g = wrap_idx(i0 - H + (t - l * R), n);
                    const int64_t o = g + (int64_t)l * n;
                    if (g >= rlo && g < rhi) return ldg(own_src + o);
                    return xf.b ? fma(xf.beta, ldg(xf.b + o), ldg(xf.a + o)) : ldg(xf.a + o);
                },
                [&](int t, double v) {
                    const int l = fdiv(t, invR);
                    Xs[l * ldx + (t - l * R)] = v;
                });
        }
        __syncthreads();
        if (single) {
            // halo rows 0..H-1 and H+n..R-1 from the staged rows
            const int nh = R - n;
            const float invh = __frcp_rn((float)max(nh, 1));
            for (int t = tid; t < nh * rc; t += WG) {
                const int l = fdiv(t, invh), j = t - l * nh;
                const int ir = j < H ? j : j + n;
                Xs[l * ldx + ir] = Xs[l * ldx + H + wrap_idx(ir - H, n)];
            }
            if (any_r1) {
                for (int b = 0; b < nblk; ++b) {
                    if (comps[b].kind != CP_OP_RANK1) continue;
                    const double* w = comps[b].data + n;
                    for (int l = wave; l < rc; l += NWAVES) {
                        double acc = 0.0;
                        for (int i = lane; i < n; i += 64) acc = fma(ldg(w + i), Xs[l * ldx + H + i], acc);
                        acc = wave_sum(acc);
                        if (lane == 0) s.dots[b * rc + l] = acc;
                    }
                }
            }
        }
        // Kt block 0 (or every block)
        const int nkb = allk ? nblk : 1;
        if (hit) {
            // kept from an earlier product of this solve
        } else if (rc == rc4) {
            // Kt rows (blk rc + k) are contiguous in memory and land at row (blk rc4 + k) of
            // the staged layout; columns j >= r of a tile only reach outputs that are dropped
            const float invr = __frcp_rn((float)r);
            auto ld = [&](int t) { return ldg(Kt + t); };
            auto st = [&](int t, double v) {
                const int row = fdiv(t, invr);
                KtS[row * LDB + (t - row * r)] = v;
            };
            if (allk) batched_loop<24>(nkb * rc * r, ld, st);
            else batched_loop<8>(nkb * rc * r, ld, st);
        } else {
            constexpr int TW = TN * 16;
            const int per = rc4 * TW;
            const float invper = __frcp_rn((float)per);
            batched_loop<4>(
                nkb * per,
                [&](int t) {
                    const int b = fdiv(t, invper), e = t - b * per;
                    const int k = e / TW, j = e - k * TW;
                    return (k < rc && j < r) ? ldg(Kt + j + (int64_t)(b * rc + k) * r) : 0.0;
                },
                [&](int t, double v) {
                    const int b = fdiv(t, invper), e = t - b * per;
                    KtS[b * ktsz + (e / TW) * LDB + e % TW] = v;
                });
        }
        Tile<F32> acc[SPW][TN];
#pragma unroll
        for (int u = 0; u < SPW; ++u)
#pragma unroll
            for (int t = 0; t < TN; ++t) acc[u][t].zero();
        // stencil coefficients of the pass rows for operator block b, CfS[buf][j][row]; a
        // thread holds at most PFC of them between the load and the LDS store
        constexpr int PFC = (CG_TAPS * NWAVES * SPW * 16 + WG - 1) / WG;
        const float invRP = __frcp_rn((float)RP);
        auto load_cf = [&](int b, double (&cv)[PFC]) {
            const int kind = comps[b].kind, h = comps[b].hbw;
            const double* data = comps[b].data;
            const bool band = kind == CP_OP_BAND;
            const int nt = (band && h <= 2) ? 2 * h + 1 : 1;
#pragma unroll
            for (int u = 0; u < PFC; ++u) {
                const int t = tid + u * WG;
                const int j = fdiv(t, invRP), i = i0 + (t - j * RP);
                double c = 0.0;
                if (j < nt && i < n && !(band && h > 2)) c = (kind == CP_OP_IDENTITY) ? 1.0 : ldg(data + (int64_t)j * n + i);
                cv[u] = c;
            }
        };
        auto store_cf = [&](int buf, const double (&cv)[PFC]) {
#pragma unroll
            for (int u = 0; u < PFC; ++u) {
                const int t = tid + u * WG;
                if (t < CG_TAPS * RP) CfS[buf * CG_TAPS * RP + t] = cv[u];
            }
        };
        if (hit) {
        } else if (allk) {
            const int per = CG_TAPS * RP;
            const float invper = __frcp_rn((float)per);
            batched_loop<4>(
                nblk * per,
                [&](int t) {
                    const int b = fdiv(t, invper), e = t - b * per;
                    const int j = fdiv(e, invRP), i = i0 + (e - j * RP);
                    const int kind = comps[b].kind, h = comps[b].hbw;
                    const bool band = kind == CP_OP_BAND;
                    const int nt = (band && h <= 2) ? 2 * h + 1 : 1;
                    if (!(j < nt && i < n && !(band && h > 2))) return 0.0;
                    return (kind == CP_OP_IDENTITY) ? 1.0 : ldg(comps[b].data + (int64_t)j * n + i);
                },
                [&](int t, double v) { CfS[t] = v; });
        } else {
            double cv[PFC];
            load_cf(0, cv);
            store_cf(0, cv);
        }
        __syncthreads();
        // One strip and every block staged with taps of at most 5: the k-steps of all blocks
        // (blk, ks) are dealt to the waves in equal contiguous shares.  A wave gathers the
        // operands of KC steps at once (B fragments, taps, coefficients), then issues their
        // matrix-core steps back to back; the partial tiles meet below as in the block split.
        const bool flat = G == NWAVES && nsp == 1 && flat_ok;
        if (flat) {
            const int spb = rc4 >> 2;                 // k-steps per block
            const int T = nblk * spb;
            const int s0 = (wave * T) / NWAVES, s1 = ((wave + 1) * T) / NWAVES;
            const float invspb = __frcp_rn((float)spb);
            // KC steps from c0 (those at or past s1 are skipped), stencils of up to TAPS taps;
            // the staged coefficients of taps past a block's own are zero
            auto chunk = [&](int c0, auto kc_c, auto taps_c) {
                constexpr int KC = decltype(kc_c)::value;
                constexpr int TAPS = decltype(taps_c)::value;
                double bv[KC][TN], xv[KC][TAPS], cv[KC][TAPS];
                bool lv[KC];
#pragma unroll
                for (int u = 0; u < KC; ++u) {
                    const int st = min(c0 + u, s1 - 1);
                    const int blk = fdiv(st, invspb), ks = (st - blk * spb) * 4;
                    const int nt = s.bnt[blk], off0 = s.boff[blk];
                    const int l = min(ks + kq, rc - 1);
                    lv[u] = c0 + u < s1 && ks + kq < rc;
#pragma unroll
                    for (int t = 0; t < TN; ++t) bv[u][t] = KtS[blk * ktsz + (ks + kq) * LDB + t * 16 + cc];
                    const double* xr = Xs + l * ldx + cc + off0;
                    const double* cr = CfS + blk * CG_TAPS * RP + cc;
#pragma unroll
                    for (int j = 0; j < TAPS; ++j) {
                        xv[u][j] = xr[min(j, nt - 1)];
                        cv[u][j] = cr[j * RP];
                    }
                }
#pragma unroll
                for (int u = 0; u < KC; ++u) {
                    if (c0 + u < s1) {
                        double a = 0.0;
#pragma unroll
                        for (int j = 0; j < TAPS; ++j) a = fma(cv[u][j], xv[u][j], a);
                        a = lv[u] ? a : 0.0;
#pragma unroll
                        for (int t = 0; t < TN; ++t) acc[0][t].step(bv[u][t], a);
                    }
                }
            };
            auto run = [&](auto taps_c) {
                constexpr int KC = TN == 4 ? 4 : 8;
                int c0 = s0;
                for (; c0 + KC <= s1; c0 += KC) chunk(c0, std::integral_constant<int, KC>{}, taps_c);
                for (; c0 < s1; c0 += 2) chunk(c0, std::integral_constant<int, 2>{}, taps_c);
            };
            if (flat_taps == 1) run(std::integral_constant<int, 1>{});
            else if (flat_taps == 3) run(std::integral_constant<int, 3>{});
            else run(std::integral_constant<int, 5>{});
        }
        for (int blk = flat ? nblk : kg; blk < nblk; blk += G) {
            const int cur = allk ? blk : (blk & 1);
            const bool more = !allk && blk + 1 < nblk;
            double pf[PF], pc[PFC];
            if (more) {
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int t = tid + u * WG;
                    const int k = t / (TN * 16), j = t - k * (TN * 16);
                    pf[u] = (k < rc && j < r) ? ldg(Kt + j + (int64_t)((blk + 1) * rc + k) * r) : 0.0;
                }
                load_cf(blk + 1, pc);
            }
            const int kind = ufirst(comps[blk].kind);
            const int h = ufirst(comps[blk].hbw);
            const double* data = comps[blk].data;
            const bool r1 = kind == CP_OP_RANK1;
            const bool band = kind == CP_OP_BAND;
            const bool fast = !band || h <= 2;
            const int nt = band ? 2 * h + 1 : 1;
            const int off0 = band ? H - h : H;
            const double* bsrc = KtS + cur * ktsz;
            double cf[SPW][CG_TAPS];
#pragma unroll
            for (int u = 0; u < SPW; ++u)
#pragma unroll
                for (int j = 0; j < CG_TAPS; ++j)
                    cf[u][j] = (j < nt && wstrip + NWAVES * u < nsp) ? CfS[(cur * CG_TAPS + j) * RP + (wstrip + NWAVES * u) * 16 + cc] : 0.0;
            // one k-step: every lane forms the A elements of its strips (all LDS reads of the
            // step in flight together), then the matrix-core steps.  The tap count is fixed per
            // operator block, so the loop is instantiated per stencil width.
            auto ksteps = [&](auto ntap_c) {
                constexpr int NTAP = decltype(ntap_c)::value;
                constexpr int NV = NTAP > 0 ? NTAP : 1;
                // operands of one k-step: B fragments and the taps of every strip
                auto load_step = [&](int ks, double (&b)[TN], double (&xv)[SPW][NV]) {
                    const int l = min(ks + kq, rc - 1);
#pragma unroll
                    for (int t = 0; t < TN; ++t) b[t] = bsrc[(ks + kq) * LDB + t * 16 + cc];
#pragma unroll
                    for (int u = 0; u < SPW; ++u) {
                        if (NTAP == 0) {
                            xv[u][0] = s.dots[blk * rc + l];   // rank-1 block: m_i (w^T X[:, l])
                        } else if (NTAP > 0) {
                            const double* xr = Xs + l * ldx + (wstrip + NWAVES * u) * 16 + cc + off0;
#pragma unroll
                            for (int j = 0; j < NV; ++j) xv[u][j] = xr[j];
                        } else {
                            const int strip = wstrip + NWAVES * u;
                            const int i = i0 + strip * 16 + cc;
                            double v = 0.0;
                            if (i < n && strip < nsp) {
                                const double* xr = Xs + l * ldx + strip * 16 + cc + off0;
                                for (int j = 0; j < nt; ++j) v = fma(ldg(data + (int64_t)j * n + i), xr[j], v);
                            }
                            xv[u][0] = v;
                        }
                    }
                };
                double bc[TN], xc[SPW][NV];
                load_step(0, bc, xc);
                for (int ks = 0; ks < rc4; ks += 4) {
                    // the next step's LDS reads are issued before this step's matrix-core work
                    double bn[TN], xn[SPW][NV];
                    load_step(min(ks + 4, rc4 - 4), bn, xn);
                    const bool lv = ks + kq < rc;
#pragma unroll
                    for (int u = 0; u < SPW; ++u) {
                        double a = 0.0;
                        if (NTAP > 0) {
#pragma unroll
                            for (int j = 0; j < NV; ++j) a = fma(cf[u][j], xc[u][j], a);
                        } else if (NTAP == 0) {
                            a = cf[u][0] * xc[u][0];
                        } else {
                            a = xc[u][0];
                        }
                        a = lv ? a : 0.0;
                        if (wstrip + NWAVES * u < nsp) {
                            // operands swapped: the tile holds out^T, so a lane's four results
                            // are four columns of sixteen consecutive rows (coalesced stores)
#pragma unroll
                            for (int t = 0; t < TN; ++t) acc[u][t].step(bc[t], a);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < TN; ++t) bc[t] = bn[t];
#pragma unroll
                    for (int u = 0; u < SPW; ++u)
#pragma unroll
                        for (int j = 0; j < NV; ++j) xc[u][j] = xn[u][j];
                }
            };
            if (r1) ksteps(std::integral_constant<int, 0>{});
            else if (!fast) ksteps(std::integral_constant<int, -1>{});
            else if (nt == 1) ksteps(std::integral_constant<int, 1>{});
            else if (nt == 3) ksteps(std::integral_constant<int, 3>{});
            else ksteps(std::integral_constant<int, 5>{});
            if (more) {
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int t = tid + u * WG;
                    if (t < rc4 * TN * 16) {
                        const int k = t / (TN * 16), j = t - k * (TN * 16);
                        KtS[(cur ^ 1) * ktsz + k * LDB + j] = pf[u];
                    }
                }
                store_cf(cur ^ 1, pc);
            }
            if (!allk) __syncthreads();
        }
        bool done = false;
        if (flat) {
            // every wave's partial tiles through LDS; wave w adds value w of every lane and tile
            // over the waves in the order 0..3 (the order of the block split below) and
            // finishes those outputs, so the epilogue is spread over the four waves
            double* red = keep ? s.scratch + ldx * rc : KtS;
            __syncthreads();
#pragma unroll
            for (int t = 0; t < TN; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[((wave * TN + t) * 4 + v) * 64 + lane] = acc[0][t].get(v);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                double val;
                if (F32) {
                    float a = (float)red[((0 * TN + t) * 4 + wave) * 64 + lane];
#pragma unroll
                    for (int g = 1; g < NWAVES; ++g) a += (float)red[((g * TN + t) * 4 + wave) * 64 + lane];
                    val = (double)a;
                } else {
                    val = red[((0 * TN + t) * 4 + wave) * 64 + lane];
#pragma unroll
                    for (int g = 1; g < NWAVES; ++g) val += red[((g * TN + t) * 4 + wave) * 64 + lane];
                }
                const int lr = cc;
                const int col = t * 16 + Tile<F32>::row(lane, wave);
                if (lr < nrow && col < r) {
                    if (shift || dot) {
                        const double xv = Xs[col * ldx + H + lr];
                        if (shift) val = fma(lam, xv, val);
                        if (dot) part = fma(xv, val, part);
                    }
                    stg(out + (i0 + lr) + (int64_t)col * n, val);
                }
            }
            done = true;
        } else if (G > 1) {
            // partial tiles of groups 1 .. G-1 through LDS (the reduction area), added by
            // group 0 in a fixed order
            double* red = keep ? s.scratch + ldx * rc : KtS;
            __syncthreads();
            if (kg > 0 && wstrip < nsp) {
#pragma unroll
                for (int t = 0; t < TN; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        red[(((kg - 1) * nsp + wstrip) * TN + t) * 256 + v * 64 + lane] = acc[0][t].get(v);
            }
            __syncthreads();
            if (kg == 0 && wstrip < nsp) {
                for (int g = 1; g < G; ++g)
#pragma unroll
                    for (int t = 0; t < TN; ++t)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[0][t].add(v, red[(((g - 1) * nsp + wstrip) * TN + t) * 256 + v * 64 + lane]);
            }
        }
        // epilogue
#pragma unroll
        for (int u = 0; u < SPW; ++u) {
            const int strip = wstrip + NWAVES * u;
            if (strip < nsp && kg == 0 && !done) {
#pragma unroll
                for (int t = 0; t < TN; ++t) {
                    const int lr = strip * 16 + cc;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int col = t * 16 + Tile<F32>::row(lane, v);
                        if (lr < nrow && col < r) {
                            double val = acc[u][t].get(v);
                            if (shift || dot) {
                                const double xv = Xs[col * ldx + H + lr];
                                if (shift) val = fma(lam, xv, val);
                                if (dot) part = fma(xv, val, part);
                            }
                            stg(out + (i0 + lr) + (int64_t)col * n, val);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    // bookkeeping of the kept blocks: recorded, or forgotten by a product that used their space
    __syncthreads();
    if (tid_here() == 0) {
        if (keep) {
            s.kc_key = Kt;
            s.kc_base = kbase;
            s.kc_size = SA;
            s.kc_rlo = rlo;
        } else {
            s.kc_key = nullptr;
        }
    }
    return part;
}

// ------------------------------------------------------------------------------------
// Preconditioner application z = v (H_q + lambda I)^{-1} on the own rows: a row-local r x r
// product (no stencil, no halo), so plain FMA dot products from LDS replace the matrix-core
// tile machinery: Hinv (symmetric) is staged once, its loads in flight together with those
// of the transform that forms v (MODE as in xform_rows, updates of the other vectors riding
// along), then the rows in chunks of PRC.  Returns this thread's share of sum(v o z); with
// `adot`, also its share of sum(a o (a Hinv)) for the untransformed panel a in `adot_part`
// (b^T P^{-1} b of the stopping test rides along with the first residual).
// The LDS it uses lies below any operator blocks a composite product keeps across the
// solve; kept blocks it would overlap are forgotten.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ double precond_apply(const Xform& xf, int n, int r, const double* Hinv, double* out,
                                                int rlo, int rhi, bool adot, double& adot_part) {
    Smem& s = SMEM;
    constexpr int PRC = 64;                            // rows per chunk
    constexpr int HPT = (CP_MAX_RANK * CP_MAX_RANK + WG - 1) / WG;
    const int rr = r * r;
    double* Hs = s.scratch;                            // Hinv[l + j r]
    double* Xs = s.scratch + rr;                       // chunk: v[i, l] at Xs[l (PRC + 1) + i]
    const int ldx = PRC + 1;
    double* Xa = adot ? Xs + r * ldx : nullptr;        // chunk of a (with adot)
    __syncthreads();
    double hv[HPT];
#pragma unroll
    for (int u = 0; u < HPT; ++u) {
        const int t = tid_here() + u * WG;
        hv[u] = t < rr ? ldg(Hinv + t) : 0.0;
    }
    double part = 0.0, pa = 0.0;
    bool staged = false;
    for (int i0 = rlo; i0 < rhi; i0 += PRC) {
        const int nrow = min(PRC, rhi - i0);
        if (i0 > rlo) __syncthreads();
        xform_dispatch(xf, n, i0, nrow, r, true, Xs, ldx, 0, Xa);
        if (!staged) {
#pragma unroll
            for (int u = 0; u < HPT; ++u) {
                const int t = tid_here() + u * WG;
                if (t < rr) Hs[t] = hv[u];
            }
            staged = true;
        }
        __syncthreads();
        const float invr = __frcp_rn((float)nrow);
        for (int t = tid_here(); t < nrow * r; t += WG) {
            const int j = fdiv(t, invr), i = t - j * nrow;
            double acc = 0.0;
            for (int l = 0; l < r; ++l) acc = fma(Xs[l * ldx + i], Hs[l + j * r], acc);
            stg(out + (i0 + i) + (int64_t)j * n, acc);
            part = fma(Xs[j * ldx + i], acc, part);
            if (adot) {
                double acc2 = 0.0;
                for (int l = 0; l < r; ++l) acc2 = fma(Xa[l * ldx + i], Hs[l + j * r], acc2);
                pa = fma(Xa[j * ldx + i], acc2, pa);
            }
        }
    }
    adot_part = pa;
    __syncthreads();
    if (tid_here() == 0) {
        const int used = rr + (adot ? 2 : 1) * r * ldx;
        if (s.kc_key && s.kc_base < used) s.kc_key = nullptr;
    }
    return part;
}

// ------------------------------------------------------------------------------------
// balancing
// ------------------------------------------------------------------------------------

// Column norms from the panels themselves -> s.colnorm[k*r + l]
__device__ __forceinline__ void panel_colnorms() {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    const int r = pb.r;
    for (int kl = wave; kl < pb.d * r; kl += NWAVES) {
        const int k = kl / r, l = kl % r;
        const double* u = pb.U + pb.offU[k] + (int64_t)l * pb.n[k];
        double acc = 0.0;
        for (int i = lane; i < pb.n[k]; i += 64) {
            const double v = ldg(u + i);
            acc = fma(v, v, acc);
        }
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
    for (int kl = tid_here(); kl < pb.d * r; kl += WG) {
        const int k = kl / r, l = kl % r;
        const int ld = pb.mA[k] * r;
        s.colnorm[kl] = sqrt(fmax(ldg(pb.G + pb.offG[k] + (int64_t)l * ld + l), 0.0));
    }
    __syncthreads();
}

// colnorm -> scale factors (in place); a column with a zero factor keeps scale 1.
__device__ __forceinline__ void balance_scales() {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r, d = pb.d;
    for (int l = tid_here(); l < r; l += WG) {
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

// Column scaling of the panels: every row (all_rows) or the own rows of every dimension.
__device__ __forceinline__ void scale_panels(bool all_rows) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r;
    for (int k = 0; k < pb.d; ++k) {
        const int n = pb.n[k];
        int rlo = 0, rhi = n;
        if (!all_rows) own_rows(n, rlo, rhi);
        const int nown = rhi - rlo;
        double* u = pb.U + pb.offU[k];
        const float invn = __frcp_rn((float)nown);
        auto idx = [&](int t) {
            const int l = fdiv(t, invn);
            return (int64_t)(rlo + (t - l * nown)) + (int64_t)l * n;
        };
        batched_loop<8>(nown * r, [&](int t) { return ldg(u + idx(t)); },
                        [&](int t, double v) { stg(u + idx(t), v * s.colnorm[k * r + fdiv(t, invn)]); });
    }
    __syncthreads();
}

// After a sweep: rescale the Grams and cross-Grams consistently with the panels.
__device__ __forceinline__ void scale_grams(int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int r = pb.r;
    for (int k = 0; k < pb.d; ++k) {
        const int ld = pb.mA[k] * r;
        const double* sc = s.colnorm + k * r;
        double* G = pb.G + pb.offG[k];
        const float invld = __frcp_rn((float)ld), invr = __frcp_rn((float)r);
        auto modr = [&](int v) { return v - fdiv(v, invr) * r; };
        // this workgroup's slice of the entries (all of them when alone)
        const int W = ufirst(s.W), part = ufirst(s.part);
        const int ng = ld * ld, perg = (ng + W - 1) / W, g0 = min(ng, part * perg), g1 = min(ng, g0 + perg);
        batched_loop<8>(g1 - g0, [&](int t) { return ldg(G + g0 + t); },
                        [&](int t, double v) {
                            const int e = g0 + t;
                            const int j = fdiv(e, invld), i = e - j * ld;
                            stg(G + e, v * sc[modr(i)] * sc[modr(j)]);
                        });
        double* X = pb.X + pb.offX[k];
        const int nx = ld * pb.mB[k] * r0;
        const int perx = (nx + W - 1) / W, x0 = min(nx, part * perx), x1 = min(nx, x0 + perx);
        batched_loop<8>(x1 - x0, [&](int t) { return ldg(X + x0 + t); },
                        [&](int t, double v) {
                            const int e = x0 + t;
                            const int j = fdiv(e, invld), i = e - j * ld;
                            stg(X + e, v * sc[modr(i)]);
                        });
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------------
// Step residual in double-double, rank growth and term dropping (adaptive rank).  A
// problem that needs them runs on one workgroup, so every routine below covers all rows.
// ------------------------------------------------------------------------------------

// Columns of the stacked panel Z_k = [P_k | Q_k] of dimension k at ranks (r, r0): the
// applied panel P_k = [O_A^a U_k]_a (in pb.P, formed by apply_panel) and Q_k = [O_B^b V_k]_b.
__device__ __forceinline__ int stacked_cols(int k, int r, int r0) {
    const Problem& pb = SMEM.pb;
    return pb.mA[k] * r + pb.mB[k] * r0;
}

__device__ __forceinline__ const double* stacked_col(int k, int c, int r) {
    const Problem& pb = SMEM.pb;
    const int n = pb.n[k], M1 = pb.mA[k] * r;
    return c < M1 ? pb.P + (int64_t)c * n : pb.Q + pb.offQ[k] + (int64_t)(c - M1) * n;
}

// Rdd_k[i + j N] = Z_k[:, i]^T Z_k[:, j] by compensated dot products (Dot2), stored as
// (hi, lo).  Rows are staged through LDS in chunks (column c at Zs[c ld + j]); every thread
// keeps EB entries over all rows.  P_k must have been formed.
__device__ __forceinline__ void gram_dd(int k, int r, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[k], N = stacked_cols(k, r, r0);
    const int RB = min(64, SCRATCH / N - 1);
    const int ld = RB + 1;
    double* Zs = s.scratch;
    double* out = pb.Rdd + 2 * pb.offR[k];
    constexpr int EB = 8;
    const int NN = N * N;
    const float invN = __frcp_rn((float)N);
    for (int e0 = 0; e0 < NN; e0 += EB * WG) {
        double sh[EB], sc[EB];
        int ei[EB], ej[EB];
#pragma unroll
        for (int u = 0; u < EB; ++u) {
            sh[u] = sc[u] = 0.0;
            const int e = min(e0 + tid_here() + u * WG, NN - 1);
            ej[u] = fdiv(e, invN);
            ei[u] = e - ej[u] * N;
        }
        for (int i0 = 0; i0 < n; i0 += RB) {
            const int nr = min(RB, n - i0);
            const float invnr = __frcp_rn((float)nr);
            __syncthreads();
            batched_loop<4>(
                nr * N,
                [&](int t) {
                    const int c = fdiv(t, invnr);
                    return ldg(stacked_col(k, c, r) + i0 + (t - c * nr));
                },
                [&](int t, double v) {
                    const int c = fdiv(t, invnr);
                    Zs[c * ld + (t - c * nr)] = v;
                });
            __syncthreads();
            for (int j = 0; j < nr; ++j) {
#pragma unroll
                for (int u = 0; u < EB; ++u) dot2_step(Zs[ei[u] * ld + j], Zs[ej[u] * ld + j], sh[u], sc[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < EB; ++u) {
            const int e = e0 + tid_here() + u * WG;
            if (e < NN) {
                const dd v = dot2_result(sh[u], sc[u]);
                stg(out + 2 * (int64_t)e, v.hi);
                stg(out + 2 * (int64_t)e + 1, v.lo);
            }
        }
    }
    __syncthreads();
}

// Workgroup sum of two dd values in a fixed order (every thread gets the result).
__device__ __forceinline__ void wg_sum_dd2(dd& a, dd& b) {
    Smem& s = SMEM;
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    a = dd_wave_sum(a);
    b = dd_wave_sum(b);
    __syncthreads();
    if (lane == 0) {
        s.scratch[4 * wave + 0] = a.hi;
        s.scratch[4 * wave + 1] = a.lo;
        s.scratch[4 * wave + 2] = b.hi;
        s.scratch[4 * wave + 3] = b.lo;
    }
    __syncthreads();
    dd x{0.0, 0.0}, y{0.0, 0.0};
    for (int w = 0; w < NWAVES; ++w) {
        x = dd_add(x, dd{s.scratch[4 * w + 0], s.scratch[4 * w + 1]});
        y = dd_add(y, dd{s.scratch[4 * w + 2], s.scratch[4 * w + 3]});
    }
    __syncthreads();
    a = x;
    b = y;
}

// rho = ||A f - g|| / ||g||, g = B f_n, f the factors U at rank r, f_n the factors V at rank
// r0 (Q must hold [O_B^b V_k]_b).  The residual is the CP tensor with the stacked terms
//   s < TA:  eta_e  prod_k O_A^{a(e,k)} U_k      (width r, columns a(e,k) r of Z_k)
//   s >= TA: -zeta_z prod_k O_B^{b(z,k)} V_k     (width r0, columns mA_k r + b(z,k) r0)
// so ||R||^2 = sum_{s,s'} c_s c_s' sum_{l,l'} prod_k Rdd_k[col(s,k) + l, col(s',k) + l'],
// every product and sum in double-double; ||g||^2 is the part with s, s' >= TA.
__device__ __forceinline__ double step_residual(int r, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d;
    for (int k = 0; k < d; ++k) {
        const int n = pb.n[k];
        apply_panel(pb.opA[k], pb.mA[k], n, r, pb.U + pb.offU[k], pb.P, 0, n);
        gram_dd(k, r, r0);
    }
    const int TA = pb.TA, S = pb.TA + pb.TB;
    // stacked-term table in LDS: coefficient, width, first column per dimension
    double* coefS = s.scratch + 64;
    int32_t* colS = reinterpret_cast<int32_t*>(coefS + S);
    for (int t = tid_here(); t < S; t += WG) {
        const PairRec* tr = t < TA ? pb.termA + t : pb.termB + (t - TA);
        coefS[t] = t < TA ? ldg(&tr->coef) : -ldg(&tr->coef);
        const uint64_t sw = (uint64_t)__double_as_longlong(ldg(reinterpret_cast<const double*>(tr) + 1));
        for (int k = 0; k < d; ++k) {
            const int a = (int)((sw >> (8 * k)) & 0xffu);
            colS[t * CP_MAX_DIMS + k] = t < TA ? a * r : pb.mA[k] * r + a * r0;
        }
    }
    __syncthreads();
    dd num{0.0, 0.0}, den{0.0, 0.0};
    for (int sa = 0; sa < S; ++sa) {
        const int wa = sa < TA ? r : r0;
        for (int sb = 0; sb < S; ++sb) {
            const int wb = sb < TA ? r : r0;
            const double ca = coefS[sa], cb = coefS[sb];
            const bool gpart = sa >= TA && sb >= TA;
            const float inva = __frcp_rn((float)wa);
            for (int p = tid_here(); p < wa * wb; p += WG) {
                const int lp = fdiv(p, inva), l = p - lp * wa;
                dd prod{1.0, 0.0};
                for (int k = 0; k < d; ++k) {
                    const int N = stacked_cols(k, r, r0);
                    const int64_t e = (int64_t)(colS[sa * CP_MAX_DIMS + k] + l) +
                                      (int64_t)(colS[sb * CP_MAX_DIMS + k] + lp) * N;
                    const double* g = pb.Rdd + 2 * (pb.offR[k] + e);
                    prod = dd_mul(prod, dd{ldg(g), ldg(g + 1)});
                }
                prod = dd_mul_d(dd_mul_d(prod, ca), cb);
                num = dd_add(num, prod);
                if (gpart) den = dd_add(den, prod);
            }
        }
    }
    wg_sum_dd2(num, den);
    const double nv = fmax(num.hi + num.lo, 0.0), dv = den.hi + den.lo;
    return dv > 0.0 ? sqrt(nv / dv) : sqrt(nv);
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in counter form: the output for the state
// seed + (counter + 1) * gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// cv_k = t_k^T Z_k (one wave per column, rows strided by lane) and gnrm[k] = t_k^T t_k;
// P_k must hold dimension k's applied panel.
__device__ __forceinline__ void growth_contract(int k, int r, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int n = pb.n[k], N = stacked_cols(k, r, r0);
    const int lane = tid_here() & 63, wave = tid_here() >> 6;
    const double* t = pb.tv + pb.offT[k];
    double* cv = pb.cv + pb.offCv[k];
    for (int c = wave; c <= N; c += NWAVES) {
        const double* z = c < N ? stacked_col(k, c, r) : t;
        double acc = 0.0;
        for (int i = lane; i < n; i += 64) acc = fma(ldg(t + i), ldg(z + i), acc);
        acc = wave_sum(acc);
        if (lane == 0) {
            if (c < N) stg(cv + c, acc);
            else s.gnrm[k] = acc;
        }
    }
    __syncthreads();
}

// The term appended when the rank grows from r: three sweeps of rank-1 ALS fitting the
// residual tensor R = g - A f (g = B f_n), from the seeded start
// t_k[i] = 2 u - 1, u = splitmix64(seed, ((step 64 + r) 8 + k) 2^32 + i) / 2^64 (top 53 bits),
// k > 0 (dimension 0 is updated first, so its start is never read).  Update of dimension q:
//   t_q = (sum_c Z_q[:, c] beta[c]) / prod_{k != q} t_k^T t_k, with
//   beta[a r + l]          = -sum_{e: a(e,q) = a} eta_e  prod_{k != q} cv_k[a(e,k) r + l]
//   beta[mA r + b r0 + l0] =  sum_{z: b(z,q) = b} zeta_z prod_{k != q} cv_k[mA_k r + b(z,k) r0 + l0]
// (the exact minimiser of ||R - t|| over t_q).  The result becomes column r of every U_k.
__device__ __forceinline__ void grow_term(int step, int r, int r0) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d;
    for (int k = 0; k < d; ++k) {
        double* t = pb.tv + pb.offT[k];
        const uint64_t base = (((uint64_t)step * 64u + (uint64_t)r) * 8u + (uint64_t)k) << 32;
        for (int i = tid_here(); i < pb.n[k]; i += WG) {
            double v = 0.0;
            if (k > 0) v = 2.0 * ((double)(splitmix64(pb.seed, base + (uint64_t)i) >> 11) * 0x1.0p-53) - 1.0;
            stg(t + i, v);
        }
    }
    __syncthreads();
    for (int k = 1; k < d; ++k) {
        apply_panel(pb.opA[k], pb.mA[k], pb.n[k], r, pb.U + pb.offU[k], pb.P, 0, pb.n[k]);
        growth_contract(k, r, r0);
    }
    const int TA = pb.TA, TB = pb.TB;
    for (int sweep = 0; sweep < 3; ++sweep) {
        for (int q = 0; q < d; ++q) {
            const int n = pb.n[q], N = stacked_cols(q, r, r0), M1 = pb.mA[q] * r;
            double* beta = s.scratch;
            for (int c = tid_here(); c < N; c += WG) {
                const bool aside = c < M1;
                const int blk = aside ? c / r : (c - M1) / r0;
                const int l = aside ? c - blk * r : (c - M1) - blk * r0;
                const int T = aside ? TA : TB;
                double acc = 0.0;
                for (int e = 0; e < T; ++e) {
                    const PairRec* tr = aside ? pb.termA + e : pb.termB + e;
                    const uint64_t sw = (uint64_t)__double_as_longlong(ldg(reinterpret_cast<const double*>(tr) + 1));
                    if ((int)((sw >> (8 * q)) & 0xffu) != blk) continue;
                    double prod = ldg(&tr->coef);
                    for (int k = 0; k < d; ++k) {
                        if (k == q) continue;
                        const int a = (int)((sw >> (8 * k)) & 0xffu);
                        const int col = aside ? a * r + l : pb.mA[k] * r + a * r0 + l;
                        prod *= ldg(pb.cv + pb.offCv[k] + col);
                    }
                    acc += prod;
                }
                beta[c] = aside ? -acc : acc;
            }
            double nn = 1.0;
            for (int k = 0; k < d; ++k)
                if (k != q) nn *= s.gnrm[k];
            apply_panel(pb.opA[q], pb.mA[q], n, r, pb.U + pb.offU[q], pb.P, 0, n);   // ends with a barrier
            double* t = pb.tv + pb.offT[q];
            const double inv = nn > 0.0 ? 1.0 / nn : 0.0;
            for (int i = tid_here(); i < n; i += WG) {
                double acc = 0.0;
                for (int c = 0; c < N; ++c) acc = fma(ldg(stacked_col(q, c, r) + i), beta[c], acc);
                stg(t + i, nn > 0.0 ? acc * inv : 0.0);
            }
            __syncthreads();
            growth_contract(q, r, r0);
        }
    }
    // column r of every factor
    for (int k = 0; k < d; ++k) {
        const double* t = pb.tv + pb.offT[k];
        double* u = pb.U + pb.offU[k] + (int64_t)r * pb.n[k];
        for (int i = tid_here(); i < pb.n[k]; i += WG) stg(u + i, ldg(t + i));
    }
    __syncthreads();
}

// Drops the terms of weight prod_k ||U_k[:, l]|| below 1e-14 of the largest (rank
// reduction of Section 3.2); the kept columns move to the front in order, at least one is
// kept.  Returns the new rank.
__device__ __forceinline__ int drop_small_terms(int r) {
    Smem& s = SMEM;
    const Problem& pb = s.pb;
    const int d = pb.d;
    panel_colnorms();
    int32_t* keep = reinterpret_cast<int32_t*>(s.scratch);
    if (tid_here() == 0) {
        auto weight = [&](int l) {
            double p = 1.0;
            for (int k = 0; k < d; ++k) p *= s.colnorm[k * r + l];
            return p;
        };
        double wmax = 0.0;
        for (int l = 0; l < r; ++l) wmax = fmax(wmax, weight(l));
        int kept = 0;
        for (int l = 0; l < r; ++l)
            if (!(wmax > 0.0) || weight(l) >= 1e-14 * wmax) keep[1 + kept++] = l;
        if (kept == 0) keep[1 + kept++] = 0;
        keep[0] = kept;
    }
    __syncthreads();
    const int kept = keep[0];
    for (int j = 0; j < kept; ++j) {
        const int l = keep[1 + j];
        if (l == j) continue;
        for (int k = 0; k < d; ++k) {
            const int n = pb.n[k];
            double* u = pb.U + pb.offU[k];
            for (int i = tid_here(); i < n; i += WG) stg(u + i + (int64_t)j * n, ldg(u + i + (int64_t)l * n));
        }
        __syncthreads();
    }
    return kept;
}

// ------------------------------------------------------------------------------------
// the persistent kernel
// ------------------------------------------------------------------------------------
enum : int { OP_STEP, OP_REFRESH, OP_UPDATE, OP_CG, OP_DELTA, OP_JACOBI, OP_SWEEP, OP_RANK, OP_REPORT, OP_DONE };
// phases of one dimension update's composite products
enum : int { PH_RHS, PH_MV_X, PH_PRE_R0, PH_MV_P0, PH_PRE_R, PH_MV_P };

__global__ void __launch_bounds__(WG) als_persistent(const Problem* __restrict__ problems, int count, int W,
                                                      const int32_t* __restrict__ wg_first, int nx) {
    Smem& s = SMEM;
    // problem pid is advanced by its workgroups wg_first[pid] .. wg_first[pid + 1] - 1 (a
    // table of count + 1 offsets) or, without the table, by the workgroups of slots
    // pid W .. pid W + W - 1.  With nx > 1 the slots are striped over nx XCDs: the dispatcher
    // deals workgroup b to XCD b mod nx, so slot (b mod nx) (grid / nx) + b / nx puts each
    // cluster on one XCD (whether it really is there is checked at run time).
    int pid, cpart, Wp;
    if (wg_first) {
        const int b = blockIdx.x;
        int lo = 0, hi = count;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (wg_first[mid] <= b) lo = mid;
            else hi = mid;
        }
        pid = lo;
        cpart = b - wg_first[lo];
        Wp = wg_first[lo + 1] - wg_first[lo];
    } else {
        int b = blockIdx.x;
        if (nx > 1) b = (b % nx) * (int)(gridDim.x / nx) + b / nx;
        pid = b / W;
        cpart = b - pid * W;
        Wp = W;
    }
    if (pid >= count) return;
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(problems + pid);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&s.pb);
        for (int t = tid_here(); t < (int)(sizeof(Problem) / 4); t += WG) dst[t] = src[t];
        if (tid_here() == 0) {
            s.ident.kind = CP_OP_IDENTITY;
            s.ident.hbw = 0;
            s.ident.data = nullptr;
            s.part = cpart;
            s.W = Wp;
            s.bar_target = 0;
            s.sync_ok = 1;
            s.xlocal = 0;
            s.dcount = 0;
            s.kc_key = nullptr;
            // this workgroup's copy of the assembled blocks

        }
    }
    __syncthreads();
    detect_xcd_local();
    const Problem& pb = s.pb;
    const int d = ufirst(pb.d);
    int r = ufirst(pb.r);   // the current rank (changes only in adaptive mode)
    const int n_steps = ufirst(pb.n_steps), max_sweeps = ufirst(pb.max_sweeps);
    const bool mixed = pb.precision == CP_PREC_MIXED;
    // mixed-precision form: sweeps with FP32 contractions until the increment reaches the
    // FP32 floor (or the sweep budget is nearly spent), then the Grams again in FP64 and FP64
    // sweeps until eps_conv <= tol, as the plain method (with tol = 0 the caller asks for
    // exactly max_sweeps sweeps: FP32 until the last one)
    const double tol_low = pb.tol > 0.0 ? fmax(pb.tol, 1e-6) : 0.0;

    int op = OP_STEP;
    int step = 0, r0 = 0, q = 0, k = 0, k_end = 0, after = OP_UPDATE, sw = 1, ph = PH_RHS, it = 0;
    int pcg_iters = 0;
    uint32_t flags = 0;
    bool lowp = false;
    double lam = 0.0, bz = 0.0, stop = 0.0, rz = 0.0, pw = 0.0, alpha = 0.0, beta = 0.0;
    double dmax2 = 0.0, eps = 0.0, fnorm = 0.0;
    bool inc_bad = false;         // a non-finite increment this sweep (fmax would drop it)
    double eps_low_min = 1e300;   // smallest increment of the FP32 sweeps of this step
    int low_stall = 0;            // FP32 sweeps since that minimum last improved
    int psel = 0;   // which of the two search-direction buffers holds p
    int sweeps_done = 0;          // sweeps of the earlier solves of this step (rank growth)
    int low_sweeps = 0;           // sweeps of this step with FP32 contractions
    int grown = r;                // rank before the drop of negligible terms
    double rho = -1.0;            // step residual (when formed)
    bool carry = false;           // a share of ||Delta f_q||^2 waits for the next refresh's barrier
    double carry_val = 0.0;
    // the current rank into the LDS descriptor, which the routines read
    auto set_rank = [&](int rn) {
        __syncthreads();
        if (tid_here() == 0) s.pb.r = rn;
        __syncthreads();
        r = ufirst(rn);
    };

    while (op != OP_DONE) {
        op = ufirst(op);
        if (ufirst((int)s.sync_ok) == 0) {
            // a cluster barrier timed out: the problem is abandoned with a flag
            if (cpart == 0 && tid_here() == 0) {
                cp_als_report rep;
                rep.sweeps = sweeps_done + sw;
                rep.pcg_iters = pcg_iters;
                rep.eps_conv = eps;
                rep.fnorm = fnorm;
                rep.rel_residual = -1.0;
                rep.flags = flags | CP_FLAG_NOT_CONVERGED | CP_FLAG_SYNC_TIMEOUT;
                rep.final_rank = r;
                rep.grown_rank = r;
                rep.low_sweeps = low_sweeps;
                pb.reports[step < n_steps ? step : n_steps - 1] = rep;
            }
            break;
        }
        if (op == OP_STEP) {
            r0 = (step == 0) ? pb.r0 : r;
            if (cpart == 0) {
                if (step > 0) {
                    // f_n <- previous result (same packed layout, rank r)
                    for (int kk = 0; kk < d; ++kk) {
                        const double* src = pb.U + pb.offU[kk];
                        double* dst = pb.V + pb.offV[kk];
                        batched_loop<8>(pb.n[kk] * r, [&](int t) { return ldg(src + t); }, [&](int t, double v) { stg(dst + t, v); });
                    }
                    __syncthreads();
                }
                compute_Q_all(r0);
                panel_colnorms();
                balance_scales();
                scale_panels(true);
            }
            cluster_sync();
            lowp = mixed && max_sweeps > 1;
            eps_low_min = 1e300;
            low_stall = 0;
            pcg_iters = 0;
            sweeps_done = 0;
            low_sweeps = 0;
            rho = -1.0;
            flags = CP_FLAG_NOT_CONVERGED;
            eps = fnorm = dmax2 = 0.0;
            inc_bad = false;
            sw = 1;
            q = 0;
            k = 0;
            k_end = d;
            after = OP_UPDATE;
            op = OP_REFRESH;
        } else if (op == OP_REFRESH) {
            if (carry) {
                // dimension k was just solved: its Grams from x, with the sum of ||Delta f_k||^2
                const double d2 = ufirst(refresh_dim(k, r0, lowp, pb.vx, true, carry_val));
                inc_bad = inc_bad || !isfinite(d2);
                dmax2 = fmax(dmax2, d2);
                carry = false;
            } else {
                refresh_dim(k, r0, lowp);
            }
            ++k;
            if (k >= k_end) op = after;
        } else if (op == OP_UPDATE) {
            const double trM = assemble(q, r0);
            lam = ufirst(pb.eps_reg * trM / (double)(pb.n[q] * r));
            ph = PH_RHS;
            op = OP_CG;
        } else if (op == OP_CG) {
            const int n = ufirst(pb.n[q]);
            const int m = pb.mA[q];
            const int64_t oq = pb.offU[q];
            const bool mv = ph == PH_MV_X || ph == PH_MV_P0 || ph == PH_MV_P;
            const bool pre = ph == PH_PRE_R0 || ph == PH_PRE_R;
            const OpDev* comps = pre ? &s.ident : (mv ? pb.compAA[q] : pb.compAB[q]);
            const int nblk = pre ? 1 : (mv ? m * m : m * pb.mB[q]);
            const int rc = ph == PH_RHS ? r0 : r;
            const double* Kt = pre ? pb.Hinv + (int64_t)cpart * r * r : (mv ? pb.Cm : pb.Dm);
            double* outp = pre ? pb.vz : (mv ? pb.vw : pb.vb);
            double* pcur = psel ? pb.vp2 : pb.vp;
            double* pnxt = psel ? pb.vp : pb.vp2;
            int rlo, rhi;
            own_rows(n, rlo, rhi);
            Xform xf{nullptr, nullptr, 0.0, nullptr, nullptr, nullptr, 0.0, nullptr};
            switch (ph) {
                case PH_RHS: xf.a = pb.V + pb.offV[q]; break;
                case PH_MV_X: xf.a = pb.U + oq; xf.wv = pb.vx; break;                 // x <- U_q
                case PH_PRE_R0: xf.a = pb.vb; xf.b = pb.vw; xf.beta = -1.0; xf.wv = pb.vr; break;  // r = b - A x
                case PH_MV_P0: xf.a = pb.vz; xf.wv = pcur; break;                     // p = z
                case PH_PRE_R:                                                        // r -= alpha w, x += alpha p
                    xf.a = pb.vr; xf.b = pb.vw; xf.beta = -alpha; xf.wv = pb.vr;
                    xf.x2 = pb.vx; xf.p2 = pcur; xf.alpha2 = alpha;
                    break;
                default: xf.a = pb.vz; xf.b = pcur; xf.beta = beta; xf.wv = pnxt; break;  // p' = z + beta p
            }
            const bool dot = ph != PH_RHS && ph != PH_MV_X;
            const bool f32 = lowp && !pre;
            const int tn = (r + 15) >> 4;
            double part, part_b = 0.0;
            if (pre) {
                part = precond_apply(xf, n, r, Kt, outp, rlo, rhi, ph == PH_PRE_R0, part_b);
            } else if (f32) {
                if (tn == 1) part = cgemm<true, 1>(n, r, comps, nblk, rc, xf, Kt, outp, lam, mv, dot, rlo, rhi, mv);
                else if (tn == 2) part = cgemm<true, 2>(n, r, comps, nblk, rc, xf, Kt, outp, lam, mv, dot, rlo, rhi, mv);
                else part = cgemm<true, 4>(n, r, comps, nblk, rc, xf, Kt, outp, lam, mv, dot, rlo, rhi, mv);
            } else {
                if (tn == 1) part = cgemm<false, 1>(n, r, comps, nblk, rc, xf, Kt, outp, lam, mv, dot, rlo, rhi, mv);
                else if (tn == 2) part = cgemm<false, 2>(n, r, comps, nblk, rc, xf, Kt, outp, lam, mv, dot, rlo, rhi, mv);
                else part = cgemm<false, 4>(n, r, comps, nblk, rc, xf, Kt, outp, lam, mv, dot, rlo, rhi, mv);
            }
            // dot products are summed over the cluster (fixed order); b^T P^{-1} b of the stopping
            // test is summed with r^T P^{-1} r of the first residual
            double val;
            if (ph == PH_PRE_R0) {
                double sv, su;
                const double bpart = wg_sum(part_b, s.red);
                cluster_sum2(wg_sum(part, s.red), bpart, sv, su);
                val = ufirst(sv);
                bz = ufirst(su);
            } else {
                val = ufirst(dot ? cluster_sum(wg_sum(part, s.red)) : wg_sum(part, s.red));
            }
            if (ph == PH_MV_P) psel ^= 1;   // the new direction is now the current one
            bool finish = false;
            switch (ph) {
                case PH_RHS:
                    // the new update's blocks and preconditioner: nothing kept is valid
                    if (tid_here() == 0) s.kc_key = nullptr;
                    flags |= factor_precond(lam);
                    psel = 0;
                    ph = PH_MV_X;
                    break;
                case PH_MV_X:
                    ph = PH_PRE_R0;
                    break;
                case PH_PRE_R0: {
                    // Stopping test in the preconditioned (energy-like) norm:
                    // r^T P^{-1} r <= tol^2 b^T P^{-1} b.  Since P ~ J_q^T J_q it bounds the
                    // change of the represented tensor, also along near-singular directions.
                    // FP32 contractions cannot resolve the system below ~1e-7; the FP64
                    // sweeps finish it.
                    rz = val;
                    const double ptol = lowp ? fmax(pb.pcg_tol, 1e-6) : pb.pcg_tol;
                    stop = ptol * ptol * bz;
                    it = 0;
                    if (rz <= stop) finish = true;
                    else ph = PH_MV_P0;
                    break;
                }
                case PH_MV_P0:
                case PH_MV_P:
                    pw = val;
                    ++it;
                    alpha = rz / pw;
                    ph = PH_PRE_R;
                    break;
                case PH_PRE_R: {
                    const double rzn = val;
                    if (rzn <= stop || !(pw > 0.0)) {
                        finish = true;
                    } else if (it >= pb.pcg_max) {
                        flags |= CP_FLAG_PCG_MAXITER;
                        finish = true;
                    } else {
                        beta = rzn / rz;
                        rz = rzn;
                        ph = PH_MV_P;
                    }
                    break;
                }
                default: break;
            }
            if (finish) {
                pcg_iters += it;
                op = OP_DELTA;
            }
        } else if (op == OP_DELTA) {
            // ||Delta f_q||^2 = sum((dU^T dU) o H0), dU = x - U_q; then U_q <- x (own rows).  A
            // Jacobi sweep keeps x in Unew_q instead: every dimension of the sweep is solved from
            // the factors at its start, and the Grams are refreshed once at its end.
            const int n = pb.n[q];
            double* Uq = pb.U + pb.offU[q];
            double* Udst = pb.jacobi ? pb.Unew + pb.offU[q] : Uq;
            int rlo, rhi;
            own_rows(n, rlo, rhi);
            // the own rows' share of sum_i dU_i H0 dU_i^T (dU = x - U_q, written to the free
            // panel vw; H0 symmetric): the quadratic form of the preconditioner apply
            // the staging of the apply also writes x to Udst (own rows): U_q <- x, or Unew_q
            Xform dxf{pb.vx, Uq, -1.0, pb.vw, nullptr, nullptr, 0.0, Udst};
            double unused;
            const double part = precond_apply(dxf, n, r, pb.H0, pb.vz, rlo, rhi, false, unused);
            // the workgroups' shares of ||Delta f_q||^2 are summed in a fixed order: in a Jacobi
            // sweep here (the barrier also publishes Unew_q); in a Gauss-Seidel sweep behind the
            // first barrier of the Gram refresh of dimension q, which reads x (published by the
            // last barrier of the solve) instead of U_q
            const double wpart = wg_sum(part, s.red);
            if (pb.jacobi) {
                const double d2 = ufirst(cluster_sum(wpart));
                inc_bad = inc_bad || !isfinite(d2);
                dmax2 = fmax(dmax2, d2);
                q = q + 1;
                op = (q < d) ? OP_UPDATE : OP_JACOBI;
            } else {
                carry = true;
                carry_val = wpart;
                k = q;
                k_end = q + 1;
                after = (q + 1 < d) ? OP_UPDATE : OP_SWEEP;
                q = q + 1;
                op = OP_REFRESH;
            }
        } else if (op == OP_JACOBI) {
            // end of a Jacobi sweep (Appendix B, Algorithm 1): every factor moves by the damping
            // fraction of its change, U_k <- U_k + damping (Unew_k - U_k) (own rows); the barrier
            // publishes the new factors, then every Gram is refreshed
            const double w = pb.damping;
            for (int kk = 0; kk < d; ++kk) {
                const int n = pb.n[kk];
                int rlo, rhi;
                own_rows(n, rlo, rhi);
                const int nown = rhi - rlo;
                double* Uk = pb.U + pb.offU[kk];
                const double* Nk = pb.Unew + pb.offU[kk];
                const float invn = __frcp_rn((float)nown);
                auto idx = [&](int t) {
                    const int l = fdiv(t, invn);
                    return (int64_t)(rlo + (t - l * nown)) + (int64_t)l * n;
                };
                batched_loop<8>(nown * r, [&](int t) { return ldg(Nk + idx(t)); }, [&](int t, double v) {
                    const int64_t o = idx(t);
                    const double u = ldg(Uk + o);
                    stg(Uk + o, fma(w, v - u, u));
                });
            }
            cluster_sync();
            k = 0;
            k_end = d;
            after = OP_SWEEP;
            op = OP_REFRESH;
        } else if (op == OP_SWEEP) {
            // ||f||^2 = sum o_k U_k^T U_k
            double part = 0.0;
            for (int t = tid_here(); t < r * r; t += WG) {
                const int l = t % r, lp = t / r;
                double prod = 1.0;
#pragma unroll
                for (int kk = 0; kk < CP_MAX_DIMS; ++kk)
                    if (kk < d) prod *= ldg(pb.G + pb.offG[kk] + (int64_t)lp * (pb.mA[kk] * r) + l);
                part += prod;
            }
            const double f2 = ufirst(wg_sum(part, s.red));
            fnorm = sqrt(fmax(f2, 0.0));
            const double dmax = sqrt(fmax(dmax2, 0.0));
            eps = fnorm > 0.0 ? dmax / fnorm : dmax;
            gram_colnorms();
            balance_scales();
            cluster_sync();   // every workgroup has read G before any of them rescales it
            scale_panels(false);
            scale_grams(r0);
            cluster_sync();
            const bool was_low = lowp;
            if (was_low) ++low_sweeps;
            bool refresh_all = false;
            bool done = false;
            if (inc_bad || !isfinite(f2) || !isfinite(eps)) {
                flags |= CP_FLAG_NONFINITE;
                done = true;
            } else if (was_low) {
                // the FP32 sweeps stall at their rounding floor: no new minimum (by 10 %) of
                // the increment for three sweeps ends them as well
                if (eps < 0.9 * eps_low_min) {
                    eps_low_min = eps;
                    low_stall = 0;
                } else {
                    ++low_stall;
                }
                if (eps <= tol_low || low_stall >= 3 || sw + 1 >= max_sweeps) {
                    // switch to FP64: recompute every Gram in FP64, then the refinement sweep
                    lowp = false;
                    refresh_all = true;
                }
            } else if (eps <= pb.tol) {
                flags &= ~CP_FLAG_NOT_CONVERGED;
                done = true;
            }
            if (done || sw >= max_sweeps) {
                op = pb.report_residual ? OP_RANK : OP_REPORT;
            } else {
                ++sw;
                q = 0;
                dmax2 = 0.0;
                inc_bad = false;
                if (refresh_all) {
                    k = 0;
                    k_end = d;
                    after = OP_UPDATE;
                    op = OP_REFRESH;
                } else {
                    op = OP_UPDATE;
                }
            }
        } else if (op == OP_RANK) {
            // the step residual (double-double); adaptive rank: grow while it is above tau
            // (or below the replayed rank), else drop the negligible terms
            rho = step_residual(r, r0);
            const bool adapt = pb.rank_mode == CP_RANK_ADAPTIVE;
            const bool want = pb.replay_rank >= 0 ? r < pb.replay_rank : rho > pb.tau_rank;
            if (adapt && want && r < pb.rcap && !(flags & CP_FLAG_NONFINITE)) {
                grow_term(step, r, r0);
                set_rank(r + 1);
                sweeps_done += sw;
                // solve again from the current factors (the new column balanced with the rest)
                panel_colnorms();
                balance_scales();
                scale_panels(true);
                lowp = mixed && max_sweeps > 1;
                eps_low_min = 1e300;
                low_stall = 0;
                flags = CP_FLAG_NOT_CONVERGED;
                eps = fnorm = dmax2 = 0.0;
                inc_bad = false;
                sw = 1;
                q = 0;
                k = 0;
                k_end = d;
                after = OP_UPDATE;
                op = OP_REFRESH;
            } else {
                grown = r;
                if (adapt) set_rank(drop_small_terms(r));
                op = OP_REPORT;
            }
        } else {   // OP_REPORT
            if (cpart == 0 && tid_here() == 0) {
                cp_als_report rep;
                rep.sweeps = sweeps_done + sw;
                rep.pcg_iters = pcg_iters;
                rep.eps_conv = eps;
                rep.fnorm = fnorm;
                rep.rel_residual = rho;
                rep.flags = flags;
                rep.final_rank = r;
                rep.grown_rank = pb.report_residual ? grown : r;
                rep.low_sweeps = low_sweeps;
                pb.reports[step] = rep;
            }
            if (pb.traj && cpart == 0) {
                // step s at traj + s sum_k n_k rcap, dimension after dimension (n_k x rcap,
                // the first r columns written)
                double* dst = pb.traj + (int64_t)step * [&] {
                    int64_t tot = 0;
                    for (int kk = 0; kk < d; ++kk) tot += (int64_t)pb.n[kk] * pb.rcap;
                    return tot;
                }();
                int64_t o = 0;
                for (int kk = 0; kk < d; ++kk) {
                    const int64_t cnt = (int64_t)pb.n[kk] * r;
                    for (int64_t t = tid_here(); t < cnt; t += WG) stg(dst + o + t, ldg(pb.U + pb.offU[kk] + t));
                    o += (int64_t)pb.n[kk] * pb.rcap;
                }
            }
            __syncthreads();
            ++step;
            op = (step < n_steps) ? OP_STEP : OP_DONE;
        }
    }
}

// The step residual alone (cp_residual): U holds f, V holds f_n; one workgroup.
__global__ void __launch_bounds__(WG) residual_kernel(const Problem* __restrict__ problem) {
    Smem& s = SMEM;
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(problem);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&s.pb);
        for (int t = tid_here(); t < (int)(sizeof(Problem) / 4); t += WG) dst[t] = src[t];
        if (tid_here() == 0) {
            s.ident.kind = CP_OP_IDENTITY;
            s.ident.hbw = 0;
            s.ident.data = nullptr;
            s.part = 0;
            s.W = 1;
            s.bar_target = 0;
            s.sync_ok = 1;
            s.xlocal = 0;
            s.dcount = 0;
            s.kc_key = nullptr;
        }
    }
    __syncthreads();
    const Problem& pb = s.pb;
    compute_Q_all(pb.r0);
    const double rho = step_residual(pb.r, pb.r0);
    if (tid_here() == 0) {
        cp_als_report rep;
        rep.sweeps = 0;
        rep.pcg_iters = 0;
        rep.eps_conv = 0.0;
        rep.fnorm = 0.0;
        rep.rel_residual = rho;
        rep.flags = 0;
        rep.final_rank = pb.r;
        rep.grown_rank = pb.r;
        rep.low_sweeps = 0;
        pb.reports[0] = rep;
    }
}

hipError_t launch_residual(const Problem* d_problem, hipStream_t stream) {
    hipError_t e = hipFuncSetAttribute((const void*)residual_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sizeof(Smem));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_kernel, dim3(1), dim3(WG), sizeof(Smem), stream, d_problem);
    return hipGetLastError();
}

size_t als_smem_bytes() { return sizeof(Smem); }

hipError_t prepare_als() {
    return hipFuncSetAttribute((const void*)als_persistent, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sizeof(Smem));
}

// The kernel's LDS size must have been allowed by prepare_als (launch_als does both).
// Uniform clusters of W workgroups (wg_first null), or per-problem clusters given by the
// device table wg_first (count + 1 offsets, grid = total workgroups).  Uniform clusters of
// 2 .. XCD_CUS workgroups are striped so that each lies on one XCD: the grid is XCDS
// columns of ceil(count / XCDS) clusters (the slots past count exit at once).  A row of
// XCDS clusters is at most XCDS XCD_CUS workgroups, which the device holds at once, so a
// cluster whose members are dispatched late waits only for clusters that can finish.
hipError_t launch_als_prepared(const Problem* d_problems, int count, int W, const int32_t* wg_first, int total_wg,
                               hipStream_t stream) {
    const bool stripe = !wg_first && W > 1 && W <= XCD_CUS;
    const int grid = wg_first ? total_wg : stripe ? XCDS * ((count + XCDS - 1) / XCDS) * W : count * W;
    hipLaunchKernelGGL(als_persistent, dim3(grid), dim3(WG), sizeof(Smem), stream, d_problems, count, W, wg_first,
                       stripe ? XCDS : 1);
    return hipGetLastError();
}

hipError_t launch_als(const Problem* d_problems, int count, int W, const int32_t* wg_first, int total_wg,
                      hipStream_t stream) {
    hipError_t e = prepare_als();
    if (e != hipSuccess) return e;
    return launch_als_prepared(d_problems, count, W, wg_first, total_wg, stream);
}

}  // namespace cpals
