// Internal descriptors shared by the host side of libcpals and its HIP kernels.
#pragma once
#include <stdint.h>
#include "../../include/cpals.h"

namespace cpals {

constexpr int WG = 256;           // threads of the persistent ALS workgroup (4 waves: one per SIMD,
                                  // so each wave may hold 512 registers, accumulators in AGPRs)
constexpr int NWAVES = WG / 64;

// Device scratch of the allocation-free scalar product (cp_inner_noalloc), per GPU.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;

// One distinct 1-D operator on the device.
struct OpDev {
    int32_t kind;      // cp_op_kind
    int32_t hbw;       // half bandwidth (band)
    const double* data;  // device pointer into the problem blob (null for identity)
};

// Pair record (e, z) for the Hadamard assembly of one block of C (or D) of dimension q:
// the product coefficient and, for the j-th dimension k != q (increasing k), the index
// a + b * mA[k] of the block (a, b) of G_k (or X_k) that it multiplies in.
// The same record holds one term of an operator (termA / termB): coef eta_e and, for
// every dimension k, the index of its distinct 1-D operator.
struct PairRec {
    double coef;
    uint8_t slot[CP_MAX_DIMS];
};

// Everything one ALS problem needs on the device (lives in device memory; copied to LDS
// by the kernel).
struct Problem {
    int32_t d, r, r0, n_steps;
    int32_t n[CP_MAX_DIMS];
    int32_t mA[CP_MAX_DIMS];   // distinct ops of A per dim (op 0 is the identity)
    int32_t mB[CP_MAX_DIMS];
    OpDev opA[CP_MAX_DIMS][CP_MAX_OPS];
    OpDev opB[CP_MAX_DIMS][CP_MAX_OPS];
    double trOO[CP_MAX_DIMS][CP_MAX_OPS * CP_MAX_OPS];  // <O^a, O^b>_F of A's ops, dim q
    // composite operators of dimension q: compAA[q][a + b mA] = (O_A^a)^T O_A^b,
    // compAB[q][a + b mA] = (O_A^a)^T O_B^b (band, diagonal, identity or rank-1)
    OpDev compAA[CP_MAX_DIMS][CP_MAX_OPS * CP_MAX_OPS];
    OpDev compAB[CP_MAX_DIMS][CP_MAX_OPS * CP_MAX_OPS];
    // Hadamard pair lists, per q: C blocks (mA x mA, column-major block index a + b*mA),
    // then D blocks (mA x mB, index a + b*mA).  *_off[q][blk] .. *_off[q][blk+1].
    const PairRec* pairsC;
    const PairRec* pairsD;
    int32_t offC[CP_MAX_DIMS][CP_MAX_OPS * CP_MAX_OPS + 1];
    int32_t offD[CP_MAX_DIMS][CP_MAX_OPS * CP_MAX_OPS + 1];
    // staging strides of the assembly: max_{k != q} mA[k]^2 and max_{k != q} mA[k] mB[k]
    int32_t MMq[CP_MAX_DIMS], MXq[CP_MAX_DIMS];
    // state (device, doubles): offsets in elements from the base pointers
    double* U;  int64_t offU[CP_MAX_DIMS];   // n_k x r
    double* V;  int64_t offV[CP_MAX_DIMS];   // n_k x r0
    double* Q;  int64_t offQ[CP_MAX_DIMS];   // n_k x (mB_k r0): [O_B^b V_k]_b
    double* G;  int64_t offG[CP_MAX_DIMS];   // (mA_k r)^2: P_k^T P_k
    double* X;  int64_t offX[CP_MAX_DIMS];   // (mA_k r) x (mB_k r0): P_k^T Q_k
    // scratch
    double* P;     // n_max x mA_max r  (applied panel / matvec T)
    double* Z;     // n_max x mA_max r  (matvec Z, RHS Y)
    double* Cm;    // r x (mA^2 r): Cm[l + (blk r + l') r] = C^{blk}[l, l'], blk = a + b mA
    double* Dm;    // r x (mA mB r0): Dm[l + (blk r0 + l0) r] = D^{blk}[l, l0]
    double* H0;    // r x r
    double* Hinv;  // r x r
    double* vb; double* vx; double* vr; double* vz; double* vp; double* vw;  // n_max x r
    // options
    double tol, eps_reg, pcg_tol;
    int32_t max_sweeps, pcg_max, precision, pad_;
    // rank control: r above is the rank the first step starts from; every panel holds rcap
    // columns (rcap = r in fixed mode)
    int32_t rcap, rank_mode, replay_rank, report_residual;
    double tau_rank;
    uint64_t seed;
    // sweeps: Gauss-Seidel (jacobi 0) or damped Jacobi, whose new factors wait in Unew
    // (offsets offU) until the sweep's end
    int32_t jacobi, pad2_;
    double damping;
    double* Unew;
    // the operators' terms (residual and growth): coef, and per dimension the op index
    int32_t TA, TB;
    const PairRec* termA;
    const PairRec* termB;
    // step residual in double-double: Grams of the stacked panel [P_k | Q_k] of dimension k,
    // entry e as (hi, lo) at Rdd[2 (offR[k] + e)]
    double* Rdd;  int64_t offR[CP_MAX_DIMS];
    // growth term: t_k (n_k) at tv + offT[k]; t_k^T [P_k | Q_k] at cv + offCv[k]
    double* tv;   int64_t offT[CP_MAX_DIMS];
    double* cv;   int64_t offCv[CP_MAX_DIMS];
    // outputs
    cp_als_report* reports;   // device array of n_steps
    double* traj;             // nullable: n_steps * sum_k n_k r
    // cluster of W workgroups advancing this problem together (grid rows split between
    // them); W = 1: one workgroup.  Partial sums meet in device memory after a barrier.
    int32_t W, psz;           // cluster size; doubles per workgroup in the Gram partial area
    uint32_t* bar;            // arrival counter of the cluster barrier (zero at launch)
    double* gpart;            // [W][psz] Gram / cross-Gram partials
    double* dpart;            // [2][W][8] scalar partials (dot products, trace), alternating
    double* vp2;              // second search-direction buffer (p is double-buffered)
};

// Scalar product of two CP tensors: per-dimension Gram partials over row chunks.
struct GramJob {
    const double* X[CP_MAX_DIMS];
    const double* Y[CP_MAX_DIMS];
    int32_t ldx[CP_MAX_DIMS], ldy[CP_MAX_DIMS];
    int32_t n[CP_MAX_DIMS];
    int32_t chunk0[CP_MAX_DIMS + 1];   // prefix sum of row chunks per dimension
    int32_t chunk_rows[CP_MAX_DIMS];   // rows per chunk (a multiple of 64)
    int32_t d, rx, ry;
};

// Operator application job.
struct ApplyJob {
    const double* X[CP_MAX_DIMS];
    double* Y[CP_MAX_DIMS];
    int32_t ldx[CP_MAX_DIMS], ldy[CP_MAX_DIMS], n[CP_MAX_DIMS];
    OpDev ops[CP_MAX_DIMS][CP_MAX_OPS];
    const double* coef;       // device, n_terms
    const int32_t* op_index;  // device, n_terms x d
    int32_t d, r, n_terms;
};

}  // namespace cpals
