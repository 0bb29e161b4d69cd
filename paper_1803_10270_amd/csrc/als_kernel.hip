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

namespace cpals {

struct Smem {
    Problem pb;
    double red[2 * NWAVES];
    double dots[CP_MAX_OPS * CP_MAX_RANK];
    double chol[CP_MAX_RANK * CP_MAX_RANK];
    double linv[CP_MAX_RANK * CP_MAX_RANK];
    double colnorm[CP_MAX_DIMS * CP_MAX_RANK];
    double scal[8];
    int32_t iscal[8];
};

// ------------------------------------------------------------------------------------
// applied panels
// ------------------------------------------------------------------------------------

// out[:, a*r:(a+1)*r] = O^a in (n x r panel, ld ldin), for the m operators ops[0..m).
__device__ void apply_ops_fwd(Smem& s, const OpDev* ops, int m, int n, int r, const double* in, int ldin,
                              double* out) {
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
__device__ double apply_ops_t_sum(Smem& s, const OpDev* ops, int m, int n, int r, const double* Z,
                                  double lam, const double* p, double* w) {
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
        const double pv = p[t];
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
// Gram refresh of one dimension: P_k = [O^a U_k], G_k = P_k^T P_k, X_k = P_k^T Q_k
// ------------------------------------------------------------------------------------
__device__ void refresh_dim(Smem& s, int k, int r0) {
    const Problem& pb = s.pb;
    const int n = pb.n[k], r = pb.r, m = pb.mA[k], mb = pb.mB[k];
    apply_ops_fwd(s, pb.opA[k], m, n, r, pb.U + pb.offU[k], n, pb.P);
    wg_gemm<true, false>(m * r, m * r, n, 1.0, pb.P, n, pb.P, n, 0.0, pb.G + pb.offG[k], m * r);
    wg_gemm<true, false>(m * r, mb * r0, n, 1.0, pb.P, n, pb.Q + pb.offQ[k], n, 0.0, pb.X + pb.offX[k], m * r);
    __syncthreads();
}

__device__ void compute_Q(Smem& s, int k, int r0) {
    const Problem& pb = s.pb;
    const int n = pb.n[k];
    apply_ops_fwd(s, pb.opB[k], pb.mB[k], n, r0, pb.V + pb.offV[k], n, pb.Q + pb.offQ[k]);
}

// ------------------------------------------------------------------------------------
// Hadamard assembly for dimension q: C (mA x mA blocks r x r), D (mA x mB blocks r x r0),
// H0 = o_{k != q} U_k^T U_k.  Returns trace(M_q) (without the shift).
// ------------------------------------------------------------------------------------
__device__ double assemble(Smem& s, int q, int r0) {
    const Problem& pb = s.pb;
    const int d = pb.d, r = pb.r, mq = pb.mA[q], mbq = pb.mB[q];
    const int ldC = mq * r;
    double trpart = 0.0;
    // C blocks
    const int rr = r * r;
    const int nC = mq * mq * rr;
    for (int t = threadIdx.x; t < nC; t += WG) {
        const int blk = t / rr, e = t % rr;
        const int l = e % r, lp = e / r;
        const int a = blk % mq, b = blk / mq;
        double acc = 0.0;
        for (int pi = pb.offC[q][blk]; pi < pb.offC[q][blk + 1]; ++pi) {
            const PairRec& pr = pb.pairsC[pi];
            double prod = pr.coef;
            for (int k = 0; k < d; ++k) {
                if (k == q) continue;
                const int ld = pb.mA[k] * r;
                prod *= pb.G[pb.offG[k] + (int64_t)(pr.b[k] * r + lp) * ld + pr.a[k] * r + l];
            }
            acc += prod;
        }
        pb.Cm[(a * r + l) + (int64_t)(b * r + lp) * ldC] = acc;
        if (l == lp) trpart = fma(acc, pb.trOO[q][blk], trpart);
    }
    // D blocks
    const int rr0 = r * r0;
    const int nD = mq * mbq * rr0;
    for (int t = threadIdx.x; t < nD; t += WG) {
        const int blk = t / rr0, e = t % rr0;
        const int l = e % r, l0 = e / r;
        const int a = blk % mq, b = blk / mq;
        double acc = 0.0;
        for (int pi = pb.offD[q][blk]; pi < pb.offD[q][blk + 1]; ++pi) {
            const PairRec& pr = pb.pairsD[pi];
            double prod = pr.coef;
            for (int k = 0; k < d; ++k) {
                if (k == q) continue;
                const int ld = pb.mA[k] * r;
                prod *= pb.X[pb.offX[k] + (int64_t)(pr.b[k] * r0 + l0) * ld + pr.a[k] * r + l];
            }
            acc += prod;
        }
        pb.Dm[(a * r + l) + (int64_t)(b * r0 + l0) * ldC] = acc;
    }
    // H0
    for (int t = threadIdx.x; t < rr; t += WG) {
        const int l = t % r, lp = t / r;
        double prod = 1.0;
        for (int k = 0; k < d; ++k) {
            if (k == q) continue;
            prod *= pb.G[pb.offG[k] + (int64_t)lp * (pb.mA[k] * r) + l];
        }
        pb.H0[t] = prod;
    }
    return wg_sum(trpart, s.red);  // includes the barrier that publishes C, D, H0
}

// ------------------------------------------------------------------------------------
// Preconditioner: Hinv = (H0 + lam I)^{-1} via Cholesky in LDS (wave 0).  Returns flags.
// ------------------------------------------------------------------------------------
__device__ uint32_t factor_precond(Smem& s, double lam) {
    const Problem& pb = s.pb;
    const int r = pb.r;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* c = s.chol;
    double* li = s.linv;
    for (int t = threadIdx.x; t < r * r; t += WG) {
        const int i = t % r, j = t / r;
        c[t] = pb.H0[t] + ((i == j) ? lam : 0.0);
    }
    __syncthreads();
    if (wave == 0) {
        double maxdiag = 0.0;
        for (int j = 0; j < r; ++j) maxdiag = fmax(maxdiag, c[j + j * r]);
        uint32_t fl = 0;
        const int i = lane;
        for (int j = 0; j < r; ++j) {
            double piv = c[j + j * r];
            // H0 + lam I is positive definite for lam > 0; a pivot at or below zero can only
            // come from rounding, and is replaced by the shift itself.
            if (!(piv > 1e-12 * maxdiag)) fl |= CP_FLAG_REGULARIZED;
            if (!(piv > 0.0)) piv = (lam > 0.0) ? lam : 1e-300;
            const double dj = sqrt(piv);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (i > j && i < r) c[i + j * r] /= dj;
            if (i == j) c[j + j * r] = dj;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (i > j && i < r) {
                const double lij = c[i + j * r];
                for (int k = j + 1; k <= i; ++k) c[i + k * r] -= lij * c[k + j * r];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        // column `lane` of L^{-1} by forward substitution (entries above the diagonal are 0)
        if (lane < r) {
            const int j = lane;
            for (int ii = 0; ii < j; ++ii) li[ii + j * r] = 0.0;
            li[j + j * r] = 1.0 / c[j + j * r];
            for (int ii = j + 1; ii < r; ++ii) {
                double acc = 0.0;
                for (int k = j; k < ii; ++k) acc = fma(c[ii + k * r], li[k + j * r], acc);
                li[ii + j * r] = -acc / c[ii + ii * r];
            }
        }
        if (lane == 0) s.iscal[0] = (int32_t)fl;
    }
    __syncthreads();
    // Hinv = L^{-T} L^{-1}
    for (int t = threadIdx.x; t < r * r; t += WG) {
        const int a = t % r, b = t / r;
        const int i0 = a > b ? a : b;
        double acc = 0.0;
        for (int i = i0; i < r; ++i) acc = fma(li[i + a * r], li[i + b * r], acc);
        pb.Hinv[t] = acc;
    }
    __syncthreads();
    return (uint32_t)s.iscal[0];
}

// ------------------------------------------------------------------------------------
// (M_q + lam I) p -> w, returns <p, w>
// ------------------------------------------------------------------------------------
__device__ double matvec(Smem& s, int q, double lam, const double* p, double* w) {
    const Problem& pb = s.pb;
    const int n = pb.n[q], r = pb.r, m = pb.mA[q];
    apply_ops_fwd(s, pb.opA[q], m, n, r, p, n, pb.P);
    // Z[:, a-block] = sum_b T_b (C^{ab})^T  ->  Z = T Cm^T
    wg_gemm<false, true>(n, m * r, m * r, 1.0, pb.P, n, pb.Cm, m * r, 0.0, pb.Z, n);
    __syncthreads();
    return apply_ops_t_sum(s, pb.opA[q], m, n, r, pb.Z, lam, p, w);
}

// z = r Hinv (each grid row multiplied by the symmetric Hinv); returns <r, z>.
__device__ double precond(Smem& s, int n, const double* rv, double* zv) {
    const Problem& pb = s.pb;
    const int r = pb.r;
    wg_gemm<false, false>(n, r, r, 1.0, rv, n, pb.Hinv, r, 0.0, zv, n);
    __syncthreads();
    double part = 0.0;
    for (int t = threadIdx.x; t < n * r; t += WG) part = fma(rv[t], zv[t], part);
    return wg_sum(part, s.red);
}

// ------------------------------------------------------------------------------------
// one dimension update; returns ||Delta f_q||^2 and accumulates pcg iterations / flags
// ------------------------------------------------------------------------------------
__device__ double update_dim(Smem& s, int q, int r0, int& pcg_iters, uint32_t& flags) {
    const Problem& pb = s.pb;
    const int n = pb.n[q], r = pb.r, m = pb.mA[q], mb = pb.mB[q];
    const int nr = n * r;
    double* Uq = pb.U + pb.offU[q];

    const double trM = assemble(s, q, r0);
    const double lam = pb.eps_reg * trM / (double)nr;

    // right-hand side b = sum_a (O^a)^T [Q_q D^T]_a
    wg_gemm<false, true>(n, m * r, mb * r0, 1.0, pb.Q + pb.offQ[q], n, pb.Dm, m * r, 0.0, pb.Z, n);
    __syncthreads();
    {
        bool any_rank1 = false;
        for (int a = 0; a < m; ++a) any_rank1 |= (pb.opA[q][a].kind == CP_OP_RANK1);
        if (any_rank1)
            for (int a = 0; a < m; ++a)
                if (pb.opA[q][a].kind == CP_OP_RANK1)
                    wg_coldots(n, r, pb.opA[q][a].data, pb.Z + (int64_t)a * r * n, n, s.dots + a * r);
        for (int a = 0; a < m; ++a) {
            if (a == 0) apply_op_t<false>(pb.opA[q][a], n, r, pb.Z, n, pb.vb, n, s.dots + a * r);
            else apply_op_t<true>(pb.opA[q][a], n, r, pb.Z + (int64_t)a * r * n, n, pb.vb, n, s.dots + a * r);
        }
        __syncthreads();
    }

    flags |= factor_precond(s, lam);

    // PCG from the current factor
    double* x = pb.vx;
    double* rv = pb.vr;
    double* z = pb.vz;
    double* p = pb.vp;
    double* w = pb.vw;
    for (int t = threadIdx.x; t < nr; t += WG) x[t] = Uq[t];
    __syncthreads();
    // Stopping test in the preconditioned (energy-like) norm: r^T P^{-1} r <= tol^2 b^T P^{-1} b.
    // Since P ~ J_q^T J_q, this bounds the change of the represented tensor, also along
    // near-singular directions of H_q where the plain residual norm says little.
    const double bz = precond(s, n, pb.vb, z);
    matvec(s, q, lam, x, w);
    for (int t = threadIdx.x; t < nr; t += WG) rv[t] = pb.vb[t] - w[t];
    __syncthreads();
    double rz = precond(s, n, rv, z);
    const double stop = pb.pcg_tol * pb.pcg_tol * bz;
    int it = 0;
    if (rz > stop) {
        for (int t = threadIdx.x; t < nr; t += WG) p[t] = z[t];
        __syncthreads();
        for (it = 1; it <= pb.pcg_max; ++it) {
            const double pw = matvec(s, q, lam, p, w);
            const double alpha = rz / pw;
            for (int t = threadIdx.x; t < nr; t += WG) {
                x[t] = fma(alpha, p[t], x[t]);
                rv[t] = fma(-alpha, w[t], rv[t]);
            }
            __syncthreads();
            const double rzn = precond(s, n, rv, z);
            if (rzn <= stop || !(pw > 0.0)) break;
            const double beta = rzn / rz;
            rz = rzn;
            for (int t = threadIdx.x; t < nr; t += WG) p[t] = fma(beta, p[t], z[t]);
            __syncthreads();
        }
        if (it > pb.pcg_max) {
            flags |= CP_FLAG_PCG_MAXITER;
            it = pb.pcg_max;
        }
    }
    pcg_iters += it;

    // ||Delta f_q||^2 = sum((dU^T dU) o H0), dU = x - U_q; then U_q <- x
    for (int t = threadIdx.x; t < nr; t += WG) w[t] = x[t] - Uq[t];
    __syncthreads();
    wg_gemm<true, false>(r, r, n, 1.0, w, n, w, n, 0.0, pb.S, r);
    for (int t = threadIdx.x; t < nr; t += WG) Uq[t] = x[t];
    __syncthreads();
    double part = 0.0;
    for (int t = threadIdx.x; t < r * r; t += WG) part = fma(pb.S[t], pb.H0[t], part);
    const double delta2 = wg_sum(part, s.red);
    refresh_dim(s, q, r0);
    return delta2;
}

// ------------------------------------------------------------------------------------
// balancing
// ------------------------------------------------------------------------------------

// Column norms from the panels themselves -> s.colnorm[k*r + l]
__device__ void panel_colnorms(Smem& s) {
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
__device__ void gram_colnorms(Smem& s) {
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
__device__ void balance_scales(Smem& s) {
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

__device__ void scale_panels(Smem& s) {
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
__device__ void scale_grams(Smem& s, int r0) {
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
    extern __shared__ unsigned char smem_raw[];
    Smem& s = *reinterpret_cast<Smem*>(smem_raw);
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
        for (int k = 0; k < d; ++k) compute_Q(s, k, r0);
        panel_colnorms(s);
        balance_scales(s);
        scale_panels(s);
        for (int k = 0; k < d; ++k) refresh_dim(s, k, r0);

        int sweeps = 0, pcg_iters = 0;
        uint32_t flags = CP_FLAG_NOT_CONVERGED;
        double eps = 0.0, fnorm = 0.0;
        for (int sw = 1; sw <= pb.max_sweeps; ++sw) {
            double dmax2 = 0.0;
            for (int q = 0; q < d; ++q) {
                const double d2 = update_dim(s, q, r0, pcg_iters, flags);
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
            gram_colnorms(s);
            balance_scales(s);
            scale_panels(s);
            scale_grams(s, r0);
            sweeps = sw;
            if (!isfinite(eps)) {
                flags |= CP_FLAG_NONFINITE;
                break;
            }
            if (eps <= pb.tol) {
                flags &= ~CP_FLAG_NOT_CONVERGED;
                break;
            }
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
