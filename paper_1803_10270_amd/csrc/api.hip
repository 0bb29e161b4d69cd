// Host side of the libcpals C ABI: argument validation, problem packing, workspace
// management and kernel launches.  See include/cpals.h for the contract of every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "cpals_internal.h"

namespace cpals {
// defined in basic_kernels.hip
int gram_chunks(const int32_t* n, int d, int32_t* chunk0, int32_t* chunk_rows, int max_chunks);
hipError_t noalloc_scratch_init(int device);
double* noalloc_scratch(int device);
hipError_t launch_inner(const GramJob& job, double* partial, double* out, bool sqrt_out, hipStream_t st);
hipError_t launch_apply(const ApplyJob& job, int max_n, hipStream_t st);
// defined in als_kernel.hip
hipError_t launch_als(const Problem* d_problems, int count, int W, const int32_t* wg_first, int total_wg,
                      hipStream_t stream);
hipError_t prepare_als();
hipError_t launch_als_prepared(const Problem* d_problems, int count, int W, const int32_t* wg_first, int total_wg,
                               hipStream_t stream);
size_t als_smem_bytes();
hipError_t launch_residual(const Problem* d_problem, hipStream_t stream);
}  // namespace cpals

using namespace cpals;

struct cp_batch_plan_s;

struct cp_handle_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int max_cluster = 16;     // workgroups that may share one problem (cp_set_cluster)
    int n_cu = 256;           // compute units of the device (co-residency bound of clusters)
    std::map<std::string, int> tuned;   // cluster size per problem shape (cp_tune_cluster)
    std::string err;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_user = false;     // ws is the caller's (cp_set_workspace): never reallocated
};

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

cp_status fail(cp_handle h, cp_status st, const std::string& msg) {
    if (h) h->err = msg;
    return st;
}

cp_status hip_fail(cp_handle h, hipError_t e, const char* what) {
    return fail(h, CP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                     \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return hip_fail(h, e_, what); \
    } while (0)

// The handle's workspace holds at least `bytes`.  A library-owned workspace grows (the
// stream is drained first: its old contents are not kept); a caller-owned one is never
// reallocated, and a request beyond its size is CP_ERR_WORKSPACE.
cp_status ensure_ws(cp_handle h, size_t bytes) {
    if (bytes <= h->ws_bytes) return CP_OK;
    if (h->ws_user)
        return fail(h, CP_ERR_WORKSPACE, "workspace too small: the call needs " + std::to_string(bytes) +
                                             " bytes, cp_set_workspace gave " + std::to_string(h->ws_bytes));
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (h->ws) {
        HIP_TRY(hipFree(h->ws), "hipFree");
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    size_t sz = std::max(bytes, (size_t)1 << 20);
    HIP_TRY(hipMalloc(&h->ws, sz), "hipMalloc(workspace)");
    h->ws_bytes = sz;
    return CP_OK;
}

bool adaptive(const cp_als_opts& o) { return o.rank_mode == CP_RANK_ADAPTIVE; }
// the problem forms its step residual on the device (and then runs on one workgroup)
bool with_residual(const cp_als_opts& o) { return adaptive(o) || o.report_residual != 0; }
// columns every panel of the problem holds
int rank_capacity(const cp_tensor& f_io, const cp_als_opts& o) { return adaptive(o) ? o.rank_cap : f_io.r; }

cp_status check_tensor(cp_handle h, const cp_tensor* t, const char* name, int max_n) {
    if (!t) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + " is null");
    if (t->d < 1 || t->d > CP_MAX_DIMS) return fail(h, CP_ERR_SHAPE, std::string(name) + ": d out of range");
    if (t->r < 1 || t->r > CP_MAX_RANK) return fail(h, CP_ERR_SHAPE, std::string(name) + ": r out of range 1..64");
    for (int k = 0; k < t->d; ++k) {
        if (t->n[k] < 1 || t->n[k] > max_n)
            return fail(h, CP_ERR_SHAPE, std::string(name) + ": n[" + std::to_string(k) + "] out of range");
        if (t->ld[k] < t->n[k]) return fail(h, CP_ERR_SHAPE, std::string(name) + ": ld < n");
        if (!t->U[k]) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + ": null panel");
    }
    return CP_OK;
}

// Host-side copy of a separable operator with the identity placed at op index 0 of every
// dimension (the Hadamard factor of the identity block, o_k U_k^T U_k, is needed for the
// preconditioner and for ||f||).
struct HostOp {
    int d = 0, T = 0;
    std::vector<double> coef;
    std::vector<int> idx;                      // T x d
    int m[CP_MAX_DIMS] = {0};
    std::vector<cp_op1d> ops[CP_MAX_DIMS];
};

cp_status check_operator(cp_handle h, const cp_operator* L, const char* name, int d, const int32_t* n,
                         bool identity_first, HostOp& out) {
    if (!L) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + " is null");
    if (L->d != d) return fail(h, CP_ERR_SHAPE, std::string(name) + ": d mismatch");
    if (L->n_terms < 1 || L->n_terms > CP_MAX_TERMS) return fail(h, CP_ERR_SHAPE, std::string(name) + ": n_terms");
    if (!L->coef || !L->op_index) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + ": null table");
    out.d = d;
    out.T = L->n_terms;
    out.coef.assign(L->coef, L->coef + L->n_terms);
    out.idx.assign(L->op_index, L->op_index + (size_t)L->n_terms * d);
    for (int k = 0; k < d; ++k) {
        const int m = L->n_ops[k];
        if (m < 1 || m > CP_MAX_OPS || !L->ops[k]) return fail(h, CP_ERR_SHAPE, std::string(name) + ": n_ops");
        out.ops[k].assign(L->ops[k], L->ops[k] + m);
        for (int a = 0; a < m; ++a) {
            const cp_op1d& o = out.ops[k][a];
            if (o.n != n[k]) return fail(h, CP_ERR_SHAPE, std::string(name) + ": operator size != n");
            if (o.kind < CP_OP_IDENTITY || o.kind > CP_OP_RANK1)
                return fail(h, CP_ERR_INVALID_ARG, std::string(name) + ": bad operator kind");
            if (o.kind != CP_OP_IDENTITY && !o.data) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + ": null op data");
            if (o.kind == CP_OP_BAND && (o.half_bw < 0 || 2 * o.half_bw + 1 > 64))
                return fail(h, CP_ERR_SHAPE, std::string(name) + ": band half width out of range");
        }
        for (int e = 0; e < out.T; ++e) {
            const int a = out.idx[(size_t)e * d + k];
            if (a < 0 || a >= m) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + ": op_index out of range");
        }
        if (identity_first) {
            int id = -1;
            for (int a = 0; a < m; ++a)
                if (out.ops[k][a].kind == CP_OP_IDENTITY) { id = a; break; }
            if (id < 0) {
                if (m == CP_MAX_OPS) return fail(h, CP_ERR_SHAPE, std::string(name) + ": no room for the identity op");
                cp_op1d ident{CP_OP_IDENTITY, n[k], 0, nullptr};
                out.ops[k].insert(out.ops[k].begin(), ident);
                for (int e = 0; e < out.T; ++e) out.idx[(size_t)e * d + k] += 1;
            } else if (id > 0) {
                std::swap(out.ops[k][0], out.ops[k][id]);
                for (int e = 0; e < out.T; ++e) {
                    int& a = out.idx[(size_t)e * d + k];
                    if (a == 0) a = id;
                    else if (a == id) a = 0;
                }
            }
        }
        out.m[k] = (int)out.ops[k].size();
    }
    for (int e = 0; e < out.T; ++e)
        if (!std::isfinite(out.coef[e])) return fail(h, CP_ERR_INVALID_ARG, std::string(name) + ": non-finite coef");
    return CP_OK;
}

size_t op_data_len(const cp_op1d& o) {
    switch (o.kind) {
        case CP_OP_DIAG: return (size_t)o.n;
        case CP_OP_BAND: return (size_t)(2 * o.half_bw + 1) * o.n;
        case CP_OP_RANK1: return (size_t)2 * o.n;
        default: return 0;
    }
}

// Dense entry O[i, j] of a 1-D operator (host, for Frobenius products).
double op_entry(const cp_op1d& o, int i, int j) {
    const int n = o.n;
    switch (o.kind) {
        case CP_OP_IDENTITY: return i == j ? 1.0 : 0.0;
        case CP_OP_DIAG: return i == j ? o.data[i] : 0.0;
        case CP_OP_BAND: {
            double v = 0.0;
            for (int jj = 0; jj <= 2 * o.half_bw; ++jj) {
                int c = ((i + jj - o.half_bw) % n + n) % n;
                if (c == j) v += o.data[(size_t)jj * n + i];
            }
            return v;
        }
        default: return o.data[i] * o.data[n + j];
    }
}

// <O1, O2>_F = trace(O1^T O2).
double frob(const cp_op1d& a, const cp_op1d& b) {
    const int n = a.n;
    if (a.kind == CP_OP_RANK1 || b.kind == CP_OP_RANK1) {
        if (a.kind == CP_OP_RANK1 && b.kind == CP_OP_RANK1) {
            double s1 = 0.0, s2 = 0.0;
            for (int i = 0; i < n; ++i) { s1 += a.data[i] * b.data[i]; s2 += a.data[n + i] * b.data[n + i]; }
            return s1 * s2;
        }
        const cp_op1d& R = (a.kind == CP_OP_RANK1) ? a : b;
        const cp_op1d& S = (a.kind == CP_OP_RANK1) ? b : a;
        // sum_ij m_i w_j S_ij over S's sparsity (S not rank-1)
        double s = 0.0;
        for (int i = 0; i < n; ++i) {
            if (S.kind == CP_OP_BAND) {
                std::vector<int> cols;
                for (int jj = 0; jj <= 2 * S.half_bw; ++jj) {
                    const int c = ((i + jj - S.half_bw) % n + n) % n;
                    if (std::find(cols.begin(), cols.end(), c) == cols.end()) cols.push_back(c);
                }
                for (int c : cols) s += R.data[i] * R.data[n + c] * op_entry(S, i, c);
            } else {
                s += R.data[i] * R.data[n + i] * op_entry(S, i, i);
            }
        }
        return s;
    }
    // both sparse (identity / diag / band): sum over the union of row patterns
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        std::vector<int> cols;
        auto add = [&](const cp_op1d& o) {
            if (o.kind == CP_OP_BAND) {
                for (int jj = 0; jj <= 2 * o.half_bw; ++jj) {
                    const int c = ((i + jj - o.half_bw) % n + n) % n;
                    if (std::find(cols.begin(), cols.end(), c) == cols.end()) cols.push_back(c);
                }
            } else if (std::find(cols.begin(), cols.end(), i) == cols.end()) {
                cols.push_back(i);
            }
        };
        add(a);
        const std::vector<int> ca = cols;
        cols.clear();
        add(b);
        for (int c : ca)
            if (std::find(cols.begin(), cols.end(), c) != cols.end()) s += op_entry(a, i, c) * op_entry(b, i, c);
    }
    return s;
}

// Sparse rows of a non-rank-1 operator: rows[i] = (column, value) with duplicates merged.
std::vector<std::vector<std::pair<int, double>>> op_rows(const cp_op1d& o) {
    const int n = o.n;
    std::vector<std::vector<std::pair<int, double>>> rows(n);
    auto add = [&](int i, int j, double v) {
        for (auto& e : rows[i])
            if (e.first == j) { e.second += v; return; }
        rows[i].push_back({j, v});
    };
    for (int i = 0; i < n; ++i) {
        switch (o.kind) {
            case CP_OP_IDENTITY: add(i, i, 1.0); break;
            case CP_OP_DIAG: add(i, i, o.data[i]); break;
            case CP_OP_BAND:
                for (int jj = 0; jj <= 2 * o.half_bw; ++jj) add(i, ((i + jj - o.half_bw) % n + n) % n, o.data[(size_t)jj * n + i]);
                break;
            default: break;
        }
    }
    return rows;
}

// y = O^T x for any operator kind (host).
std::vector<double> op_apply_t(const cp_op1d& o, const std::vector<double>& x) {
    const int n = o.n;
    std::vector<double> y(n, 0.0);
    if (o.kind == CP_OP_RANK1) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += o.data[k] * x[k];
        for (int j = 0; j < n; ++j) y[j] = o.data[n + j] * s;
        return y;
    }
    auto rows = op_rows(o);
    for (int k = 0; k < n; ++k)
        for (auto& e : rows[k]) y[e.first] += e.second * x[k];
    return y;
}

// Internal composite operator (a^T b) in the device kinds.
struct CompOp {
    int kind = CP_OP_IDENTITY;
    int hbw = 0;
    std::vector<double> data;
};

cp_status compose_t(cp_handle h, const cp_op1d& a, const cp_op1d& b, CompOp& out) {
    const int n = a.n;
    out = CompOp();
    if (a.kind == CP_OP_IDENTITY && b.kind == CP_OP_IDENTITY) return CP_OK;
    if (a.kind == CP_OP_RANK1 || b.kind == CP_OP_RANK1) {
        std::vector<double> m(n), w(n);
        if (a.kind == CP_OP_RANK1 && b.kind == CP_OP_RANK1) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += a.data[i] * b.data[i];
            for (int i = 0; i < n; ++i) { m[i] = s * a.data[n + i]; w[i] = b.data[n + i]; }
        } else if (a.kind == CP_OP_RANK1) {
            // (m_a w_a^T)^T B = w_a (B^T m_a)^T
            std::vector<double> ma(a.data, a.data + n);
            std::vector<double> bt = op_apply_t(b, ma);
            for (int i = 0; i < n; ++i) { m[i] = a.data[n + i]; w[i] = bt[i]; }
        } else {
            // A^T (m_b w_b^T) = (A^T m_b) w_b^T
            std::vector<double> mb(b.data, b.data + n);
            std::vector<double> at = op_apply_t(a, mb);
            for (int i = 0; i < n; ++i) { m[i] = at[i]; w[i] = b.data[n + i]; }
        }
        out.kind = CP_OP_RANK1;
        out.data.resize(2 * (size_t)n);
        for (int i = 0; i < n; ++i) { out.data[i] = m[i]; out.data[n + i] = w[i]; }
        return CP_OK;
    }
    auto ra = op_rows(a), rb = op_rows(b);
    std::vector<std::vector<std::pair<int, double>>> c(n);
    for (int k = 0; k < n; ++k)
        for (auto& ea : ra[k])
            for (auto& eb : rb[k]) {
                const int i = ea.first, j = eb.first;
                bool found = false;
                for (auto& e : c[i])
                    if (e.first == j) { e.second += ea.second * eb.second; found = true; break; }
                if (!found) c[i].push_back({j, ea.second * eb.second});
            }
    int hb = 0;
    bool diag = true;
    for (int i = 0; i < n; ++i)
        for (auto& e : c[i]) {
            int off = ((e.first - i) % n + n) % n;
            if (off > n / 2) off -= n;
            hb = std::max(hb, std::abs(off));
            if (e.first != i) diag = false;
        }
    if (diag) {
        out.kind = CP_OP_DIAG;
        out.data.assign(n, 0.0);
        for (int i = 0; i < n; ++i)
            for (auto& e : c[i]) out.data[i] += e.second;
        return CP_OK;
    }
    if (2 * hb + 1 > 64) return fail(h, CP_ERR_UNSUPPORTED, "composite operator bandwidth above 31");
    out.kind = CP_OP_BAND;
    out.hbw = hb;
    out.data.assign((size_t)(2 * hb + 1) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (auto& e : c[i]) {
            int off = ((e.first - i) % n + n) % n;
            if (off > n / 2) off -= n;
            out.data[(size_t)(off + hb) * n + i] += e.second;
        }
    return CP_OK;
}

// Byte layout of one problem's device region.
struct Layout {
    size_t problem, opdata, pairsC, pairsD, U, Unew, V, Q, G, X, P, Z, Cm, Dm, H0, Hinv, vec, reports, bar, gpart, dpart,
        termA, termB, Rdd, tv, cv, total;
    size_t n_opdata, n_pairsC, n_pairsD;
    int64_t offU[CP_MAX_DIMS], offV[CP_MAX_DIMS], offQ[CP_MAX_DIMS], offG[CP_MAX_DIMS], offX[CP_MAX_DIMS];
    int64_t offR[CP_MAX_DIMS], offT[CP_MAX_DIMS], offCv[CP_MAX_DIMS];
    int nmax, mAmax, mBmax, r0max, rc;
};

struct Packed {
    Problem pb;
    std::vector<double> opdata;
    std::vector<PairRec> pairsC, pairsD;
    std::vector<PairRec> termA, termB;   // the operators' terms (residual, growth)
    Layout lay;
    // host op data pointers in the same order as opdata, to rebase
    std::vector<std::pair<int, int>> opref;  // (side*CP_MAX_DIMS + k, a)
};

cp_status pack_problem(cp_handle h, const HostOp& A, const HostOp& B, const cp_tensor* f_init, const cp_tensor* f_io,
                       int n_steps, const cp_als_opts& o, int W, Packed& pk) {
    const int d = f_io->d, r = f_io->r, r0 = f_init->r;
    const int rc = rank_capacity(*f_io, o);   // every panel holds rc columns
    if (r > rc) return fail(h, CP_ERR_SHAPE, "the guess has more columns than rank_cap");
    Problem& pb = pk.pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.d = d;
    pb.r = r;
    pb.r0 = r0;
    pb.n_steps = n_steps;
    Layout& L = pk.lay;
    L.nmax = 0;
    L.mAmax = 0;
    L.mBmax = 0;
    L.rc = rc;
    L.r0max = (n_steps > 1) ? std::max(r0, rc) : r0;
    for (int k = 0; k < d; ++k) {
        pb.n[k] = f_io->n[k];
        pb.mA[k] = A.m[k];
        pb.mB[k] = B.m[k];
        L.nmax = std::max(L.nmax, pb.n[k]);
        L.mAmax = std::max(L.mAmax, A.m[k]);
        L.mBmax = std::max(L.mBmax, B.m[k]);
    }
    // operator data
    pk.opdata.clear();
    std::vector<size_t> offA[CP_MAX_DIMS], offB[CP_MAX_DIMS];
    for (int side = 0; side < 2; ++side) {
        const HostOp& X = side == 0 ? A : B;
        for (int k = 0; k < d; ++k) {
            for (int a = 0; a < X.m[k]; ++a) {
                const cp_op1d& op = X.ops[k][a];
                const size_t len = op_data_len(op);
                (side == 0 ? offA : offB)[k].push_back(pk.opdata.size());
                pk.opdata.insert(pk.opdata.end(), op.data, op.data + len);
                // keep 32-byte alignment of every array
                while (pk.opdata.size() % 4) pk.opdata.push_back(0.0);
            }
        }
    }
    // composite operators (a^T b) per dim, appended to the operator data
    std::vector<size_t> offAA[CP_MAX_DIMS], offAB[CP_MAX_DIMS];
    std::vector<int> kindAA[CP_MAX_DIMS], kindAB[CP_MAX_DIMS], hbAA[CP_MAX_DIMS], hbAB[CP_MAX_DIMS];
    for (int k = 0; k < d; ++k) {
        for (int side = 0; side < 2; ++side) {
            const HostOp& R = side == 0 ? A : B;
            for (int b = 0; b < R.m[k]; ++b)
                for (int a = 0; a < A.m[k]; ++a) {
                    CompOp co;
                    cp_status st = compose_t(h, A.ops[k][a], R.ops[k][b], co);
                    if (st != CP_OK) return st;
                    (side == 0 ? offAA : offAB)[k].push_back(pk.opdata.size());
                    (side == 0 ? kindAA : kindAB)[k].push_back(co.kind);
                    (side == 0 ? hbAA : hbAB)[k].push_back(co.hbw);
                    pk.opdata.insert(pk.opdata.end(), co.data.begin(), co.data.end());
                    while (pk.opdata.size() % 4) pk.opdata.push_back(0.0);
                }
        }
    }
    // Frobenius products of A's ops per dim
    for (int q = 0; q < d; ++q)
        for (int a = 0; a < A.m[q]; ++a)
            for (int b = 0; b < A.m[q]; ++b) pb.trOO[q][a + b * A.m[q]] = frob(A.ops[q][a], A.ops[q][b]);
    // pair lists
    pk.pairsC.clear();
    pk.pairsD.clear();
    for (int q = 0; q < d; ++q) {
        const int mq = A.m[q];
        int MM = 1, MX = 1;
        for (int k = 0; k < d; ++k)
            if (k != q) {
                MM = std::max(MM, A.m[k] * A.m[k]);
                MX = std::max(MX, A.m[k] * B.m[k]);
            }
        pb.MMq[q] = MM;
        pb.MXq[q] = MX;
        for (int blk = 0; blk < mq * mq; ++blk) {
            pb.offC[q][blk] = (int32_t)pk.pairsC.size();
            for (int e = 0; e < A.T; ++e)
                for (int z = 0; z < A.T; ++z) {
                    const int a = A.idx[(size_t)e * d + q], b = A.idx[(size_t)z * d + q];
                    if (a + b * mq != blk) continue;
                    PairRec pr;
                    std::memset(&pr, 0, sizeof(pr));
                    pr.coef = A.coef[e] * A.coef[z];
                    for (int k = 0, j = 0; k < d; ++k) {
                        if (k == q) continue;
                        pr.slot[j++] = (uint8_t)(A.idx[(size_t)e * d + k] + A.idx[(size_t)z * d + k] * A.m[k]);
                    }
                    pk.pairsC.push_back(pr);
                }
        }
        pb.offC[q][mq * mq] = (int32_t)pk.pairsC.size();
        const int mbq = B.m[q];
        for (int blk = 0; blk < mq * mbq; ++blk) {
            pb.offD[q][blk] = (int32_t)pk.pairsD.size();
            for (int e = 0; e < A.T; ++e)
                for (int z = 0; z < B.T; ++z) {
                    const int a = A.idx[(size_t)e * d + q], b = B.idx[(size_t)z * d + q];
                    if (a + b * mq != blk) continue;
                    PairRec pr;
                    std::memset(&pr, 0, sizeof(pr));
                    pr.coef = A.coef[e] * B.coef[z];
                    for (int k = 0, j = 0; k < d; ++k) {
                        if (k == q) continue;
                        pr.slot[j++] = (uint8_t)(A.idx[(size_t)e * d + k] + B.idx[(size_t)z * d + k] * A.m[k]);
                    }
                    pk.pairsD.push_back(pr);
                }
        }
        pb.offD[q][mq * mbq] = (int32_t)pk.pairsD.size();
    }
    // layout (bytes, relative to the region base)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o2 = off;
        off = align_up(off + bytes);
        return o2;
    };
    L.problem = take(sizeof(Problem));
    L.opdata = take(pk.opdata.size() * sizeof(double));
    L.pairsC = take(pk.pairsC.size() * sizeof(PairRec));
    L.pairsD = take(pk.pairsD.size() * sizeof(PairRec));
    size_t nU = 0, nV = 0, nQ = 0, nG = 0, nX = 0, nR = 0, nT = 0, nC = 0;
    const bool res = with_residual(o);
    for (int k = 0; k < d; ++k) {
        L.offU[k] = (int64_t)nU;
        nU += (size_t)pb.n[k] * rc;
        L.offV[k] = (int64_t)nV;
        nV += (size_t)pb.n[k] * L.r0max;
        L.offQ[k] = (int64_t)nQ;
        nQ += (size_t)pb.n[k] * B.m[k] * L.r0max;
        L.offG[k] = (int64_t)nG;
        nG += (size_t)(A.m[k] * rc) * (A.m[k] * rc);
        L.offX[k] = (int64_t)nX;
        nX += (size_t)(A.m[k] * rc) * (B.m[k] * L.r0max);
        // residual / growth: the stacked panel [P_k | Q_k] has mA rc + mB r0max columns
        const size_t Nk = (size_t)A.m[k] * rc + (size_t)B.m[k] * L.r0max;
        L.offR[k] = (int64_t)nR;
        L.offT[k] = (int64_t)nT;
        L.offCv[k] = (int64_t)nC;
        if (res) {
            nR += Nk * Nk;
            nT += (size_t)pb.n[k];
            nC += Nk;
        }
    }
    L.U = take(nU * 8);
    L.Unew = take(o.sweep_mode == CP_SWEEP_JACOBI ? nU * 8 : 8);
    L.V = take(nV * 8);
    L.Q = take(nQ * 8);
    L.G = take(nG * 8);
    L.X = take(nX * 8);
    L.P = take((size_t)L.nmax * L.mAmax * rc * 8);
    L.Z = take((size_t)L.nmax * L.mAmax * rc * 8);
    L.Cm = take((size_t)(L.mAmax * rc) * (L.mAmax * rc) * 8);
    L.Dm = take((size_t)(L.mAmax * rc) * (L.mBmax * L.r0max) * 8);
    L.H0 = take((size_t)rc * rc * 8);
    L.Hinv = take((size_t)W * rc * rc * 8);
    L.vec = take((size_t)7 * align_up((size_t)L.nmax * rc * 8));
    L.reports = take((size_t)n_steps * sizeof(cp_als_report));
    size_t psz = 0;
    for (int k = 0; k < d; ++k)
        psz = std::max(psz, (size_t)(A.m[k] * rc) * (A.m[k] * rc) + (size_t)(A.m[k] * rc) * (B.m[k] * L.r0max));
    pb.W = W;
    pb.psz = (int32_t)psz;
    L.bar = take(256);
    L.gpart = take(W > 1 ? (size_t)W * psz * 8 : 8);
    L.dpart = take((size_t)2 * W * 8 * 8);
    // terms of A and B (coefficient, op index per dimension)
    pk.termA.assign(A.T, PairRec{});
    pk.termB.assign(B.T, PairRec{});
    for (int side = 0; side < 2; ++side) {
        const HostOp& X = side == 0 ? A : B;
        std::vector<PairRec>& out = side == 0 ? pk.termA : pk.termB;
        for (int e = 0; e < X.T; ++e) {
            std::memset(&out[e], 0, sizeof(PairRec));
            out[e].coef = X.coef[e];
            for (int k = 0; k < d; ++k) out[e].slot[k] = (uint8_t)X.idx[(size_t)e * d + k];
        }
    }
    L.termA = take((size_t)A.T * sizeof(PairRec));
    L.termB = take((size_t)B.T * sizeof(PairRec));
    L.Rdd = take(std::max<size_t>(nR, 1) * 16);
    L.tv = take(std::max<size_t>(nT, 1) * 8);
    L.cv = take(std::max<size_t>(nC, 1) * 8);
    L.total = off;
    L.n_opdata = pk.opdata.size();
    L.n_pairsC = pk.pairsC.size();
    L.n_pairsD = pk.pairsD.size();
    // options
    pb.tol = o.tol;
    pb.eps_reg = o.eps_reg;
    pb.pcg_tol = o.pcg_tol;
    pb.max_sweeps = o.max_sweeps;
    pb.pcg_max = o.pcg_max_iter;
    pb.precision = o.precision;
    pb.rcap = rc;
    pb.rank_mode = o.rank_mode;
    pb.replay_rank = adaptive(o) ? o.replay_rank : -1;
    pb.report_residual = res ? 1 : 0;
    pb.tau_rank = o.tau_rank;
    pb.seed = o.seed;
    pb.TA = A.T;
    pb.TB = B.T;
    pb.jacobi = o.sweep_mode == CP_SWEEP_JACOBI ? 1 : 0;
    pb.damping = o.damping;
    // op descriptors get device pointers at rebase time; remember offsets in elements
    for (int k = 0; k < d; ++k) {
        for (int i = 0; i < A.m[k] * A.m[k]; ++i) {
            pb.compAA[k][i].kind = kindAA[k][i];
            pb.compAA[k][i].hbw = hbAA[k][i];
            pb.compAA[k][i].data = reinterpret_cast<const double*>(offAA[k][i]);
        }
        for (int i = 0; i < A.m[k] * B.m[k]; ++i) {
            pb.compAB[k][i].kind = kindAB[k][i];
            pb.compAB[k][i].hbw = hbAB[k][i];
            pb.compAB[k][i].data = reinterpret_cast<const double*>(offAB[k][i]);
        }
        for (int a = 0; a < A.m[k]; ++a) {
            pb.opA[k][a].kind = A.ops[k][a].kind;
            pb.opA[k][a].hbw = A.ops[k][a].half_bw;
            pb.opA[k][a].data = reinterpret_cast<const double*>(offA[k][a]);
        }
        for (int b = 0; b < B.m[k]; ++b) {
            pb.opB[k][b].kind = B.ops[k][b].kind;
            pb.opB[k][b].hbw = B.ops[k][b].half_bw;
            pb.opB[k][b].data = reinterpret_cast<const double*>(offB[k][b]);
        }
    }
    (void)h;
    return CP_OK;
}

// Fill in device pointers of a packed problem placed at device address `base`.
void rebase(Packed& pk, char* base, double* traj) {
    Problem& pb = pk.pb;
    const Layout& L = pk.lay;
    double* opd = reinterpret_cast<double*>(base + L.opdata);
    for (int k = 0; k < pb.d; ++k) {
        for (int i = 0; i < pb.mA[k] * pb.mA[k]; ++i)
            pb.compAA[k][i].data = pb.compAA[k][i].kind == CP_OP_IDENTITY ? nullptr
                                   : opd + reinterpret_cast<size_t>(pb.compAA[k][i].data);
        for (int i = 0; i < pb.mA[k] * pb.mB[k]; ++i)
            pb.compAB[k][i].data = pb.compAB[k][i].kind == CP_OP_IDENTITY ? nullptr
                                   : opd + reinterpret_cast<size_t>(pb.compAB[k][i].data);
        for (int a = 0; a < pb.mA[k]; ++a)
            pb.opA[k][a].data = pb.opA[k][a].kind == CP_OP_IDENTITY ? nullptr
                                : opd + reinterpret_cast<size_t>(pb.opA[k][a].data);
        for (int b = 0; b < pb.mB[k]; ++b)
            pb.opB[k][b].data = pb.opB[k][b].kind == CP_OP_IDENTITY ? nullptr
                                : opd + reinterpret_cast<size_t>(pb.opB[k][b].data);
        pb.offU[k] = L.offU[k];
        pb.offV[k] = L.offV[k];
        pb.offQ[k] = L.offQ[k];
        pb.offG[k] = L.offG[k];
        pb.offX[k] = L.offX[k];
        pb.offR[k] = L.offR[k];
        pb.offT[k] = L.offT[k];
        pb.offCv[k] = L.offCv[k];
    }
    pb.termA = reinterpret_cast<const PairRec*>(base + L.termA);
    pb.termB = reinterpret_cast<const PairRec*>(base + L.termB);
    pb.Rdd = reinterpret_cast<double*>(base + L.Rdd);
    pb.tv = reinterpret_cast<double*>(base + L.tv);
    pb.cv = reinterpret_cast<double*>(base + L.cv);
    pb.pairsC = reinterpret_cast<const PairRec*>(base + L.pairsC);
    pb.pairsD = reinterpret_cast<const PairRec*>(base + L.pairsD);
    pb.U = reinterpret_cast<double*>(base + L.U);
    pb.Unew = reinterpret_cast<double*>(base + L.Unew);
    pb.V = reinterpret_cast<double*>(base + L.V);
    pb.Q = reinterpret_cast<double*>(base + L.Q);
    pb.G = reinterpret_cast<double*>(base + L.G);
    pb.X = reinterpret_cast<double*>(base + L.X);
    pb.P = reinterpret_cast<double*>(base + L.P);
    pb.Z = reinterpret_cast<double*>(base + L.Z);
    pb.Cm = reinterpret_cast<double*>(base + L.Cm);
    pb.Dm = reinterpret_cast<double*>(base + L.Dm);
    pb.H0 = reinterpret_cast<double*>(base + L.H0);
    pb.Hinv = reinterpret_cast<double*>(base + L.Hinv);
    const size_t vstride = align_up((size_t)L.nmax * L.rc * 8);
    char* vb = base + L.vec;
    pb.vb = reinterpret_cast<double*>(vb + 0 * vstride);
    pb.vx = reinterpret_cast<double*>(vb + 1 * vstride);
    pb.vr = reinterpret_cast<double*>(vb + 2 * vstride);
    pb.vz = reinterpret_cast<double*>(vb + 3 * vstride);
    pb.vp = reinterpret_cast<double*>(vb + 4 * vstride);
    pb.vw = reinterpret_cast<double*>(vb + 5 * vstride);
    pb.vp2 = reinterpret_cast<double*>(vb + 6 * vstride);
    pb.reports = reinterpret_cast<cp_als_report*>(base + L.reports);
    pb.bar = reinterpret_cast<uint32_t*>(base + L.bar);
    pb.gpart = reinterpret_cast<double*>(base + L.gpart);
    pb.dpart = reinterpret_cast<double*>(base + L.dpart);
    pb.traj = traj;
}

cp_status check_opts(cp_handle h, const cp_als_opts* o) {
    if (!o) return fail(h, CP_ERR_INVALID_ARG, "opts is null");
    if (!(o->tol >= 0.0) || o->max_sweeps < 1 || !(o->eps_reg >= 0.0) || !(o->pcg_tol > 0.0) || o->pcg_max_iter < 1)
        return fail(h, CP_ERR_INVALID_ARG, "bad ALS options");
    if (o->precision != CP_PREC_FP64 && o->precision != CP_PREC_MIXED)
        return fail(h, CP_ERR_INVALID_ARG, "bad precision");
    if (o->rank_mode != CP_RANK_FIXED && o->rank_mode != CP_RANK_ADAPTIVE)
        return fail(h, CP_ERR_INVALID_ARG, "bad rank_mode");
    if (o->rank_mode == CP_RANK_ADAPTIVE &&
        (!(o->tau_rank >= 0.0) || o->rank_cap < 1 || o->rank_cap > CP_MAX_RANK || o->replay_rank > CP_MAX_RANK))
        return fail(h, CP_ERR_INVALID_ARG, "adaptive rank needs tau_rank >= 0 and 1 <= rank_cap <= CP_MAX_RANK");
    if (o->report_residual != 0 && o->report_residual != 1)
        return fail(h, CP_ERR_INVALID_ARG, "report_residual must be 0 or 1");
    if (o->sweep_mode != CP_SWEEP_GAUSS_SEIDEL && o->sweep_mode != CP_SWEEP_JACOBI)
        return fail(h, CP_ERR_INVALID_ARG, "bad sweep_mode");
    if (o->sweep_mode == CP_SWEEP_JACOBI && !(o->damping > 0.0 && o->damping <= 1.0))
        return fail(h, CP_ERR_INVALID_ARG, "Jacobi damping must be in (0, 1]");
    return CP_OK;
}


cp_status copy_panels_in(cp_handle h, hipStream_t st, const cp_tensor* t, double* dst, const int64_t* off) {
    for (int k = 0; k < t->d; ++k)
        HIP_TRY(hipMemcpy2DAsync(dst + off[k], (size_t)t->n[k] * 8, t->U[k], (size_t)t->ld[k] * 8, (size_t)t->n[k] * 8,
                                 t->r, hipMemcpyDeviceToDevice, st),
                "hipMemcpy2DAsync(in)");
    return CP_OK;
}

cp_status copy_panels_out(cp_handle h, hipStream_t st, const double* src, const int64_t* off, cp_tensor* t) {
    for (int k = 0; k < t->d; ++k)
        HIP_TRY(hipMemcpy2DAsync(t->U[k], (size_t)t->ld[k] * 8, src + off[k], (size_t)t->n[k] * 8, (size_t)t->n[k] * 8,
                                 t->r, hipMemcpyDeviceToDevice, st),
                "hipMemcpy2DAsync(out)");
    return CP_OK;
}

// Zeroes the arrival counters of the cluster barriers (a kernel rather than a memset so that
// the sequence can be captured in a graph).
__global__ void zero_words(uint32_t* p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0u;
}

// Problems packed for one launch: the static part (operator data, pair records, problem
// descriptors) is uploaded once; every run copies the panels in, launches, copies them out.
struct Staged {
    int count = 0, n_steps = 0;
    std::vector<int> W;    // workgroups per problem
    std::vector<Packed> pk;
    std::vector<size_t> base;
    size_t total = 0;      // packed regions; the descriptor array and the workgroup table follow
    size_t bytes = 0;      // total device bytes
    Problem* d_desc = nullptr;
    int32_t* d_wg_first = nullptr;   // null: every problem has W[0] workgroups
    int total_wg = 0;
    std::vector<Problem> descs;      // host copies (sources of the uploads)
    std::vector<int32_t> wg_first;
};

// Cluster size for a single problem: the largest power of two <= max_cluster with every
// n_k a multiple of 16 W (16-row strips per workgroup) and no rank-1 operator.
int cluster_size(cp_handle h, const HostOp& A, const HostOp& B, const cp_tensor& f) {
    bool ok = f.d > 1;
    for (int k = 0; k < f.d; ++k) {
        for (int a = 0; a < A.m[k]; ++a) ok = ok && A.ops[k][a].kind != CP_OP_RANK1;
        for (int b = 0; b < B.m[k]; ++b) ok = ok && B.ops[k][b].kind != CP_OP_RANK1;
    }
    if (!ok) return 1;
    int W = 1;
    while (2 * W <= std::min(h->max_cluster, 256)) W *= 2;
    for (; W > 1; W /= 2) {
        bool div = true;
        for (int k = 0; k < f.d; ++k) div = div && (f.n[k] % (16 * W) == 0);
        if (div) break;
    }
    return W;
}

// Whether W workgroups may share the problem: a power of two <= max_cluster, every n_k a
// multiple of 16 W, and (W > 1) no rank-1 operator.
bool cluster_ok(cp_handle h, const HostOp& A, const HostOp& B, const cp_tensor& f, int W) {
    if (W < 1 || (W & (W - 1)) || W > h->max_cluster) return false;
    if (W == 1) return true;
    return cluster_size(h, A, B, f) >= W;
}

// The problem shape a tuned cluster size is recorded for.
std::string shape_key(const HostOp& A, const HostOp& B, const cp_tensor& f_init, const cp_tensor& f_io,
                      const cp_als_opts& o) {
    std::string k = "d=" + std::to_string(f_io.d) + ";n=";
    for (int i = 0; i < f_io.d; ++i) k += (i ? "," : "") + std::to_string(f_io.n[i]);
    k += ";r=" + std::to_string(f_io.r) + ";r0=" + std::to_string(f_init.r) + ";mA=";
    for (int i = 0; i < f_io.d; ++i) k += (i ? "," : "") + std::to_string(A.m[i]);
    k += ";mB=";
    for (int i = 0; i < f_io.d; ++i) k += (i ? "," : "") + std::to_string(B.m[i]);
    k += ";prec=" + std::to_string((int)o.precision);
    return k;
}

// Workgroups per problem.  One problem: its tuned size when one is recorded (and still
// admissible), else the largest admissible.  Several problems: their tuned sizes (1 where
// none is recorded), provided every workgroup of the launch fits on the device at once (a
// cluster's workgroups wait for each other), else one workgroup each.
// Problems that form their step residual (adaptive rank, report_residual) keep one workgroup.
std::vector<int> choose_clusters(cp_handle h, int count, const HostOp* A, const HostOp* B, const cp_tensor* f_init,
                                 const cp_tensor* f_io, const cp_als_opts* o) {
    std::vector<int> W(count, 1);
    if (count == 1) {
        if (with_residual(o[0])) return W;
        auto it = h->tuned.find(shape_key(A[0], B[0], f_init[0], f_io[0], o[0]));
        W[0] = (it != h->tuned.end() && cluster_ok(h, A[0], B[0], f_io[0], it->second))
                   ? it->second : cluster_size(h, A[0], B[0], f_io[0]);
        return W;
    }
    if (h->tuned.empty()) return W;
    long total = 0;
    for (int i = 0; i < count; ++i) {
        auto it = h->tuned.find(shape_key(A[i], B[i], f_init[i], f_io[i], o[i]));
        if (!with_residual(o[i]) && it != h->tuned.end() && cluster_ok(h, A[i], B[i], f_io[i], it->second))
            W[i] = it->second;
        total += W[i];
    }
    if (total > h->n_cu) std::fill(W.begin(), W.end(), 1);
    return W;
}

cp_status stage_problems(cp_handle h, int count, const HostOp* A, const HostOp* B, const cp_tensor* f_init,
                         const cp_tensor* f_io, int n_steps, const cp_als_opts* o, const std::vector<int>& W,
                         Staged& S) {
    S.count = count;
    S.n_steps = n_steps;
    S.W = W;
    S.pk.resize(count);
    S.base.resize(count);
    S.total = 0;
    for (int i = 0; i < count; ++i) {
        cp_status st = pack_problem(h, A[i], B[i], &f_init[i], &f_io[i], n_steps, o[i], W[i], S.pk[i]);
        if (st != CP_OK) return st;
        S.base[i] = S.total;
        S.total += align_up(S.pk[i].lay.total);
    }
    S.bytes = S.total + align_up((size_t)count * sizeof(Problem)) + align_up((size_t)(count + 1) * sizeof(int32_t));
    return CP_OK;
}

// Rebases the packed problems onto device memory `ws` and uploads their static data and the
// descriptor array (ordered by estimated cost, largest first, so that the longest problems
// start first when workgroups outnumber CUs).
cp_status upload_static(cp_handle h, Staged& S, char* ws, double* const* traj, const cp_tensor* f_io, hipStream_t st,
                        bool wait) {
    const int count = S.count;
    std::vector<int> order(count);
    std::vector<double> cost(count);
    for (int i = 0; i < count; ++i) {
        order[i] = i;
        double c = 0.0;
        for (int k = 0; k < f_io[i].d; ++k) c += (double)f_io[i].n[k] * S.pk[i].pb.mA[k] * S.pk[i].pb.mA[k] * f_io[i].r * f_io[i].r;
        cost[i] = c;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int i = 0; i < count; ++i) {
        Packed& p = S.pk[i];
        char* b = ws + S.base[i];
        rebase(p, b, traj ? traj[i] : nullptr);
        HIP_TRY(hipMemcpyAsync(b + p.lay.opdata, p.opdata.data(), p.opdata.size() * 8, hipMemcpyHostToDevice, st),
                "hipMemcpyAsync(opdata)");
        if (!p.pairsC.empty())
            HIP_TRY(hipMemcpyAsync(b + p.lay.pairsC, p.pairsC.data(), p.pairsC.size() * sizeof(PairRec),
                                   hipMemcpyHostToDevice, st),
                    "hipMemcpyAsync(pairsC)");
        if (!p.pairsD.empty())
            HIP_TRY(hipMemcpyAsync(b + p.lay.pairsD, p.pairsD.data(), p.pairsD.size() * sizeof(PairRec),
                                   hipMemcpyHostToDevice, st),
                    "hipMemcpyAsync(pairsD)");
        HIP_TRY(hipMemcpyAsync(b + p.lay.termA, p.termA.data(), p.termA.size() * sizeof(PairRec), hipMemcpyHostToDevice,
                               st),
                "hipMemcpyAsync(termA)");
        HIP_TRY(hipMemcpyAsync(b + p.lay.termB, p.termB.data(), p.termB.size() * sizeof(PairRec), hipMemcpyHostToDevice,
                               st),
                "hipMemcpyAsync(termB)");
    }
    S.descs.resize(count);
    for (int j = 0; j < count; ++j) S.descs[j] = S.pk[order[j]].pb;
    S.d_desc = reinterpret_cast<Problem*>(ws + S.total);
    HIP_TRY(hipMemcpyAsync(S.d_desc, S.descs.data(), (size_t)count * sizeof(Problem), hipMemcpyHostToDevice, st),
            "hipMemcpyAsync(problems)");
    // workgroup table (in descriptor order) when the problems' cluster sizes differ
    bool uniform = true;
    for (int i = 1; i < count; ++i) uniform = uniform && S.W[i] == S.W[0];
    S.wg_first.assign(count + 1, 0);
    for (int j = 0; j < count; ++j) S.wg_first[j + 1] = S.wg_first[j] + S.W[order[j]];
    S.total_wg = S.wg_first[count];
    S.d_wg_first = nullptr;
    if (!uniform) {
        S.d_wg_first = reinterpret_cast<int32_t*>(ws + S.total + align_up((size_t)count * sizeof(Problem)));
        HIP_TRY(hipMemcpyAsync(S.d_wg_first, S.wg_first.data(), (size_t)(count + 1) * sizeof(int32_t),
                               hipMemcpyHostToDevice, st),
                "hipMemcpyAsync(workgroup table)");
    }
    // with `wait` the host data may be released on return (else it must outlive the copies)
    if (wait) HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    return CP_OK;
}

// One run on stream st: panels in, barrier counters zeroed (clusters), the persistent
// kernel, panels out, reports to the host buffer `rep` (count * n_steps entries).
cp_status enqueue_run(cp_handle h, const Staged& S, const cp_tensor* f_init, cp_tensor* f_io, cp_als_report* rep,
                      hipStream_t st, bool prepared = false) {
    for (int i = 0; i < S.count; ++i) {
        const Packed& p = S.pk[i];
        cp_status s2 = copy_panels_in(h, st, &f_init[i], p.pb.V, p.pb.offV);
        if (s2 != CP_OK) return s2;
        s2 = copy_panels_in(h, st, &f_io[i], p.pb.U, p.pb.offU);
        if (s2 != CP_OK) return s2;
        if (S.W[i] > 1) {
            hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, st, p.pb.bar, 64);
            HIP_TRY(hipGetLastError(), "zero_words");
        }
    }
    HIP_TRY(prepared ? launch_als_prepared(S.d_desc, S.count, S.W[0], S.d_wg_first, S.total_wg, st)
                     : launch_als(S.d_desc, S.count, S.W[0], S.d_wg_first, S.total_wg, st),
            "als kernel launch");
    for (int i = 0; i < S.count; ++i) {
        // every column the panels hold (in adaptive mode the final rank is known only from the
        // reports; the columns past it are left over from the run)
        cp_tensor out = f_io[i];
        out.r = S.pk[i].lay.rc;
        cp_status s2 = copy_panels_out(h, st, S.pk[i].pb.U, S.pk[i].pb.offU, &out);
        if (s2 != CP_OK) return s2;
        HIP_TRY(hipMemcpyAsync(rep + (size_t)i * S.n_steps, S.pk[i].pb.reports, (size_t)S.n_steps * sizeof(cp_als_report),
                               hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync(reports)");
    }
    return CP_OK;
}

cp_status check_reports(cp_handle h, const cp_als_report* reports, int n) {
    bool nc = false;
    for (int i = 0; i < n; ++i) nc |= (reports[i].flags & CP_FLAG_NOT_CONVERGED) != 0;
    if (nc) return fail(h, CP_ERR_NOT_CONVERGED, "ALS reached max_sweeps before eps_conv <= tol");
    return CP_OK;
}

// Packs, uploads and runs `count` problems (options o[i]) in the workspace from byte offset
// `base` on; in adaptive mode f_io[i].r becomes the last step's rank.
cp_status run_problems(cp_handle h, int count, const HostOp* A, const HostOp* B, const cp_tensor* f_init,
                       cp_tensor* f_io, int n_steps, const cp_als_opts* o, cp_als_report* reports, double* const* traj,
                       size_t base = 0) {
    // a problem may be shared by a cluster of workgroups (grid rows split between them)
    Staged S;
    cp_status st = stage_problems(h, count, A, B, f_init, f_io, n_steps, o,
                                  choose_clusters(h, count, A, B, f_init, f_io, o), S);
    if (st != CP_OK) return st;
    st = ensure_ws(h, base + S.bytes);
    if (st != CP_OK) return st;
    st = upload_static(h, S, static_cast<char*>(h->ws) + base, traj, f_io, h->stream, false);
    if (st != CP_OK) return st;
    st = enqueue_run(h, S, f_init, f_io, reports, h->stream);
    if (st != CP_OK) return st;
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    for (int i = 0; i < count; ++i)
        if (adaptive(o[i])) f_io[i].r = reports[(size_t)i * n_steps + n_steps - 1].final_rank;
    return check_reports(h, reports, count * n_steps);
}

// Workspace bytes of run_problems for these problems (nothing is launched).
cp_status run_bytes(cp_handle h, int count, const HostOp* A, const HostOp* B, const cp_tensor* f_init,
                    const cp_tensor* f_io, int n_steps, const cp_als_opts* o, size_t* bytes) {
    Staged S;
    cp_status st = stage_problems(h, count, A, B, f_init, f_io, n_steps, o,
                                  choose_clusters(h, count, A, B, f_init, f_io, o), S);
    if (st == CP_OK) *bytes = S.bytes;
    return st;
}

cp_status prepare_step(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_init,
                       const cp_tensor* f_io, int n_steps, const cp_als_opts* opts, HostOp& hA, HostOp& hB) {
    cp_status st = check_tensor(h, f_init, "f_init", CP_MAX_N);
    if (st != CP_OK) return st;
    st = check_tensor(h, f_io, "f_io", CP_MAX_N);
    if (st != CP_OK) return st;
    if (f_init->d != f_io->d) return fail(h, CP_ERR_SHAPE, "f_init and f_io differ in d");
    for (int k = 0; k < f_io->d; ++k)
        if (f_init->n[k] != f_io->n[k]) return fail(h, CP_ERR_SHAPE, "f_init and f_io differ in n");
    if (n_steps < 1) return fail(h, CP_ERR_INVALID_ARG, "n_steps < 1");
    st = check_opts(h, opts);
    if (st != CP_OK) return st;
    if (adaptive(*opts) && f_io->r > opts->rank_cap) return fail(h, CP_ERR_SHAPE, "f_io.r exceeds rank_cap");
    st = check_operator(h, A, "A", f_io->d, f_io->n, true, hA);
    if (st != CP_OK) return st;
    return check_operator(h, B, "B", f_io->d, f_io->n, false, hB);
}

}  // namespace

namespace cpals {
// for the other host translation units of the library (warm start)
hipStream_t handle_stream(cp_handle h) { return h->stream; }
cp_status handle_fail(cp_handle h, cp_status st, const char* msg) { return fail(h, st, msg); }
cp_status handle_check_tensor(cp_handle h, const cp_tensor* t, const char* name) {
    return check_tensor(h, t, name, CP_MAX_N);
}
}  // namespace cpals

extern "C" {

const char* cp_version(void) { return "cpals-gfx950 0.1"; }

cp_status cp_create(cp_handle* handle, void* hip_stream) {
    if (!handle) return CP_ERR_INVALID_ARG;
    cp_handle h = new (std::nothrow) cp_handle_s();
    if (!h) return CP_ERR_INVALID_ARG;
    h->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return CP_ERR_HIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && ncu > 0)
        h->n_cu = ncu;
    // the device address of this GPU's scratch array (cp_inner_noalloc), once per device
    if (noalloc_scratch_init(h->device) != hipSuccess) {
        delete h;
        return CP_ERR_HIP;
    }
    *handle = h;
    return CP_OK;
}

cp_status cp_destroy(cp_handle h) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (h->ws && !h->ws_user) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->ws);
    }
    delete h;
    return CP_OK;
}

cp_status cp_set_workspace(cp_handle h, void* dev_ptr, size_t bytes) {
    if (!h) return CP_ERR_INVALID_ARG;
    if ((!dev_ptr && bytes) || (reinterpret_cast<uintptr_t>(dev_ptr) % ALIGN) != 0)
        return fail(h, CP_ERR_INVALID_ARG, "workspace must be a 256-byte aligned device pointer (or NULL, 0)");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    if (h->ws && !h->ws_user) HIP_TRY(hipFree(h->ws), "hipFree");
    h->ws = dev_ptr;
    h->ws_bytes = dev_ptr ? bytes : 0;
    h->ws_user = dev_ptr != nullptr;
    return CP_OK;
}

cp_status cp_set_stream(cp_handle h, void* hip_stream) {
    if (!h) return CP_ERR_INVALID_ARG;
    h->stream = static_cast<hipStream_t>(hip_stream);
    return CP_OK;
}

const char* cp_last_error(cp_handle h) { return h ? h->err.c_str() : "null handle"; }

cp_status cp_set_cluster(cp_handle h, int32_t max_workgroups) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (max_workgroups < 1 || max_workgroups > 256) return fail(h, CP_ERR_INVALID_ARG, "max_workgroups must be in 1..256");
    h->max_cluster = max_workgroups;
    return CP_OK;
}

cp_status cp_als_default_opts(cp_als_opts* o) {
    if (!o) return CP_ERR_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_sweeps = 200;
    o->precision = CP_PREC_FP64;
    o->eps_reg = 1e-10;
    o->pcg_tol = 1e-14;
    o->pcg_max_iter = 100;
    o->rank_mode = CP_RANK_FIXED;
    o->tau_rank = 1e-6;
    o->rank_cap = CP_MAX_RANK;
    o->replay_rank = -1;
    o->seed = 0;
    o->report_residual = 0;
    o->sweep_mode = CP_SWEEP_GAUSS_SEIDEL;
    o->damping = 0.25;
    return CP_OK;
}

}  // extern "C"

namespace {

cp_status inner_job(cp_handle h, const cp_tensor* x, const cp_tensor* y, GramJob& job, int& nch) {
    cp_status st = check_tensor(h, x, "x", 1 << 28);
    if (st != CP_OK) return st;
    st = check_tensor(h, y, "y", 1 << 28);
    if (st != CP_OK) return st;
    if (x->d != y->d) return fail(h, CP_ERR_SHAPE, "x and y differ in d");
    std::memset(&job, 0, sizeof(job));
    job.d = x->d;
    job.rx = x->r;
    job.ry = y->r;
    for (int k = 0; k < x->d; ++k) {
        if (x->n[k] != y->n[k]) return fail(h, CP_ERR_SHAPE, "x and y differ in n");
        job.X[k] = x->U[k];
        job.Y[k] = y->U[k];
        job.ldx[k] = x->ld[k];
        job.ldy[k] = y->ld[k];
        job.n[k] = x->n[k];
    }
    nch = gram_chunks(job.n, job.d, job.chunk0, job.chunk_rows, 1 << 30);
    return CP_OK;
}

// chunk partials, then the d Grams
size_t inner_bytes(const GramJob& job, int nch) { return (size_t)(nch + job.d) * job.rx * job.ry * 8 + 256; }

cp_status inner_impl(cp_handle h, const cp_tensor* x, const cp_tensor* y, double* out_dev, bool sq, size_t base) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!out_dev) return fail(h, CP_ERR_INVALID_ARG, "out_dev is null");
    GramJob job;
    int nch = 0;
    cp_status st = inner_job(h, x, y, job, nch);
    if (st != CP_OK) return st;
    st = ensure_ws(h, base + inner_bytes(job, nch));
    if (st != CP_OK) return st;
    HIP_TRY(launch_inner(job, reinterpret_cast<double*>(static_cast<char*>(h->ws) + base), out_dev, sq, h->stream),
            "inner launch");
    return CP_OK;
}

// Operator application: the operators' data, coefficients and term table go to the host blob
// (uploaded to the workspace at `base`); the job's device pointers refer to that copy.
struct ApplyPlan {
    HostOp L;
    std::vector<double> blob;
    std::vector<size_t> offs[CP_MAX_DIMS];
    size_t coef_off = 0, idx_off_bytes = 0, bytes = 0;
};

cp_status apply_plan(cp_handle h, const cp_operator* L, const cp_tensor* x, const cp_tensor* y, ApplyPlan& P) {
    cp_status st = check_tensor(h, x, "x", 1 << 28);
    if (st != CP_OK) return st;
    st = check_operator(h, L, "L", x->d, x->n, false, P.L);
    if (st != CP_OK) return st;
    if (y) {
        if (y->d != x->d) return fail(h, CP_ERR_SHAPE, "y.d != x.d");
        if ((int64_t)y->r != (int64_t)P.L.T * x->r) return fail(h, CP_ERR_SHAPE, "y.r must equal n_terms * x.r");
        for (int k = 0; k < x->d; ++k)
            if (y->n[k] != x->n[k] || y->ld[k] < y->n[k] || !y->U[k]) return fail(h, CP_ERR_SHAPE, "bad y panel");
    }
    P.blob.clear();
    for (int k = 0; k < x->d; ++k) {
        P.offs[k].clear();
        for (int a = 0; a < P.L.m[k]; ++a) {
            const cp_op1d& op = P.L.ops[k][a];
            P.offs[k].push_back(P.blob.size());
            P.blob.insert(P.blob.end(), op.data, op.data + op_data_len(op));
            while (P.blob.size() % 4) P.blob.push_back(0.0);
        }
    }
    P.coef_off = P.blob.size();
    P.blob.insert(P.blob.end(), P.L.coef.begin(), P.L.coef.end());
    while (P.blob.size() % 4) P.blob.push_back(0.0);
    P.idx_off_bytes = P.blob.size() * 8;
    P.bytes = P.idx_off_bytes + P.L.idx.size() * 4 + 256;
    return CP_OK;
}

cp_status apply_impl(cp_handle h, const cp_operator* L, const cp_tensor* x, cp_tensor* y, size_t base) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!y) return fail(h, CP_ERR_INVALID_ARG, "y is null");
    ApplyPlan P;
    cp_status st = apply_plan(h, L, x, y, P);
    if (st != CP_OK) return st;
    st = ensure_ws(h, base + P.bytes);
    if (st != CP_OK) return st;
    char* ws = static_cast<char*>(h->ws) + base;
    HIP_TRY(hipMemcpyAsync(ws, P.blob.data(), P.blob.size() * 8, hipMemcpyHostToDevice, h->stream), "upload op data");
    HIP_TRY(hipMemcpyAsync(ws + P.idx_off_bytes, P.L.idx.data(), P.L.idx.size() * 4, hipMemcpyHostToDevice, h->stream),
            "upload op index");
    ApplyJob job;
    std::memset(&job, 0, sizeof(job));
    job.d = x->d;
    job.r = x->r;
    job.n_terms = P.L.T;
    job.coef = reinterpret_cast<const double*>(ws) + P.coef_off;
    job.op_index = reinterpret_cast<const int32_t*>(ws + P.idx_off_bytes);
    int max_n = 0;
    for (int k = 0; k < x->d; ++k) {
        job.X[k] = x->U[k];
        job.Y[k] = y->U[k];
        job.ldx[k] = x->ld[k];
        job.ldy[k] = y->ld[k];
        job.n[k] = x->n[k];
        max_n = std::max(max_n, x->n[k]);
        for (int a = 0; a < P.L.m[k]; ++a) {
            job.ops[k][a].kind = P.L.ops[k][a].kind;
            job.ops[k][a].hbw = P.L.ops[k][a].half_bw;
            job.ops[k][a].data = reinterpret_cast<const double*>(ws) + P.offs[k][a];
        }
    }
    HIP_TRY(launch_apply(job, max_n, h->stream), "apply launch");
    // the host blobs must outlive the asynchronous uploads
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return CP_OK;
}

// The identity operator on the grid of t (one term, one op per dimension).
struct IdentityOp {
    cp_op1d ident[CP_MAX_DIMS];
    double one = 1.0;
    int32_t idx[CP_MAX_DIMS] = {0};
    cp_operator I;
    explicit IdentityOp(const cp_tensor& t) {
        std::memset(&I, 0, sizeof(I));
        I.d = t.d;
        I.n_terms = 1;
        I.coef = &one;
        I.op_index = idx;
        for (int k = 0; k < t.d; ++k) {
            ident[k] = cp_op1d{CP_OP_IDENTITY, t.n[k], 0, nullptr};
            I.n_ops[k] = 1;
            I.ops[k] = &ident[k];
        }
    }
};

// The right-hand side tensor g = B f_n + c of a forced step, placed at the start of the
// workspace: its descriptor (panel k at element offset goff[k] of the workspace; until
// placed, the panel pointers name a placeholder that is never dereferenced) and byte size.
double g_placeholder;
cp_status source_tensor(cp_handle h, const cp_operator* B, const cp_tensor* f_n, const cp_tensor* source, cp_tensor& g,
                        size_t* goff, size_t& bytes) {
    cp_status st = check_tensor(h, f_n, "f_n", CP_MAX_N);
    if (st != CP_OK) return st;
    st = check_tensor(h, source, "source", CP_MAX_N);
    if (st != CP_OK) return st;
    if (!B) return fail(h, CP_ERR_INVALID_ARG, "B is null");
    if (source->d != f_n->d) return fail(h, CP_ERR_SHAPE, "source and f_n differ in d");
    for (int k = 0; k < f_n->d; ++k)
        if (source->n[k] != f_n->n[k]) return fail(h, CP_ERR_SHAPE, "source and f_n differ in n");
    const int64_t rb = (int64_t)B->n_terms * f_n->r;
    const int64_t rr = rb + source->r;
    if (B->n_terms < 1 || rr > CP_MAX_RANK)
        return fail(h, CP_ERR_SHAPE, "n_terms(B) * rank(f_n) + rank(source) exceeds CP_MAX_RANK");
    std::memset(&g, 0, sizeof(g));
    g.d = f_n->d;
    g.r = (int32_t)rr;
    size_t nel = 0;
    for (int k = 0; k < g.d; ++k) {
        g.n[k] = f_n->n[k];
        g.ld[k] = f_n->n[k];
        g.U[k] = &g_placeholder;
        goff[k] = nel;
        nel += (size_t)f_n->n[k] * rr;
    }
    bytes = align_up(nel * 8);
    return CP_OK;
}

// Residual problem: f at the U side, f_n at the V side, one step, residual only.
cp_status residual_setup(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f,
                         const cp_tensor* f_n, HostOp& hA, HostOp& hB, cp_als_opts& o) {
    cp_als_default_opts(&o);
    o.report_residual = 1;
    cp_status st = prepare_step(h, A, B, f_n, f, 1, &o, hA, hB);
    return st;
}

}  // namespace

extern "C" {

cp_status cp_inner(cp_handle h, const cp_tensor* x, const cp_tensor* y, double* out_dev) {
    return inner_impl(h, x, y, out_dev, false, 0);
}

cp_status cp_norm(cp_handle h, const cp_tensor* x, double* out_dev) { return inner_impl(h, x, x, out_dev, true, 0); }

cp_status cp_apply_operator(cp_handle h, const cp_operator* L, const cp_tensor* x, cp_tensor* y) {
    return apply_impl(h, L, x, y, 0);
}

cp_status cp_inner_noalloc(cp_handle h, const cp_tensor* x, const cp_tensor* y, double* out_dev) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!out_dev) return fail(h, CP_ERR_INVALID_ARG, "out_dev is null");
    GramJob job;
    int nch = 0;
    cp_status st = inner_job(h, x, y, job, nch);
    if (st != CP_OK) return st;
    // as many row chunks as the scratch holds partials for (beside the d Grams)
    const size_t slot = (size_t)job.rx * job.ry * 8;
    const size_t slots = (NOALLOC_SCRATCH_BYTES - 256) / slot;
    if (slots < (size_t)2 * job.d)
        return fail(h, CP_ERR_SHAPE, "cp_inner_noalloc: d * rank(x) * rank(y) exceeds the " +
                                         std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte scratch");
    nch = gram_chunks(job.n, job.d, job.chunk0, job.chunk_rows, (int)std::min<size_t>(slots - job.d, 1 << 30));
    if (inner_bytes(job, nch) > NOALLOC_SCRATCH_BYTES)
        return fail(h, CP_ERR_SHAPE, "cp_inner_noalloc: the partials exceed the scratch");
    double* scr = noalloc_scratch(h->device);
    if (!scr) return fail(h, CP_ERR_HIP, "cp_inner_noalloc: no scratch address for this device");
    HIP_TRY(launch_inner(job, scr, out_dev, false, h->stream), "inner launch");
    return CP_OK;
}

cp_status cp_als_run(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_init, cp_tensor* f_io,
                     int32_t n_steps, const cp_als_opts* opts, cp_als_report* reports, double* traj) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!reports) return fail(h, CP_ERR_INVALID_ARG, "reports is null");
    HostOp hA, hB;
    cp_status st = prepare_step(h, A, B, f_init, f_io, n_steps, opts, hA, hB);
    if (st != CP_OK) return st;
    return run_problems(h, 1, &hA, &hB, f_init, f_io, n_steps, opts, reports, traj ? &traj : nullptr);
}

cp_status cp_als_step(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n, cp_tensor* f_next,
                      const cp_als_opts* opts, cp_als_report* report) {
    return cp_als_run(h, A, B, f_n, f_next, 1, opts, report, nullptr);
}

cp_status cp_truncate(cp_handle h, const cp_tensor* g, cp_tensor* f, const cp_als_opts* opts, cp_als_report* report) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!g || !f) return fail(h, CP_ERR_INVALID_ARG, "null tensor");
    if (g->d < 1 || g->d > CP_MAX_DIMS) return fail(h, CP_ERR_SHAPE, "g: d out of range");
    IdentityOp I(*g);
    return cp_als_run(h, &I.I, &I.I, g, f, 1, opts, report, nullptr);
}

cp_status cp_als_step_source(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                             const cp_tensor* source, cp_tensor* f_next, const cp_als_opts* opts,
                             cp_als_report* report) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!source) return cp_als_step(h, A, B, f_n, f_next, opts, report);
    if (!report) return fail(h, CP_ERR_INVALID_ARG, "report is null");
    // g = B f_n + source as one CP tensor at the start of the workspace: the applied terms
    // of B f_n (coefficients in dimension 0) followed by the source's columns; the operator
    // blob of the application and the packed step follow it
    cp_tensor g;
    size_t gbytes = 0, goff[CP_MAX_DIMS];
    cp_status st = source_tensor(h, B, f_n, source, g, goff, gbytes);
    if (st != CP_OK) return st;
    IdentityOp I(g);
    HostOp hA, hB;
    st = prepare_step(h, A, &I.I, &g, f_next, 1, opts, hA, hB);
    if (st != CP_OK) return st;
    cp_tensor gb = g;
    gb.r = B->n_terms * f_n->r;
    ApplyPlan P;
    st = apply_plan(h, B, f_n, &gb, P);
    if (st != CP_OK) return st;
    size_t rbytes = 0;
    st = run_bytes(h, 1, &hA, &hB, &g, f_next, 1, opts, &rbytes);
    if (st != CP_OK) return st;
    // the whole workspace first: a library-owned one is not reallocated (emptied) midway
    st = ensure_ws(h, gbytes + std::max(P.bytes, rbytes));
    if (st != CP_OK) return st;
    for (int k = 0; k < g.d; ++k) {
        g.U[k] = static_cast<double*>(h->ws) + goff[k];
        gb.U[k] = g.U[k];
    }
    st = apply_impl(h, B, f_n, &gb, gbytes);
    if (st != CP_OK) return st;
    for (int k = 0; k < g.d; ++k)
        HIP_TRY(hipMemcpy2DAsync(g.U[k] + (size_t)gb.r * g.ld[k], (size_t)g.ld[k] * 8, source->U[k],
                                 (size_t)source->ld[k] * 8, (size_t)g.n[k] * 8, source->r, hipMemcpyDeviceToDevice,
                                 h->stream),
                "hipMemcpy2DAsync(source)");
    // A f_{n+1} = g with the identity on the right
    return run_problems(h, 1, &hA, &hB, &g, f_next, 1, opts, report, nullptr, gbytes);
}

cp_status cp_residual(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f,
                      const cp_tensor* f_n, double* rel_residual) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!A || !B || !f || !f_n || !rel_residual) return fail(h, CP_ERR_INVALID_ARG, "null argument");
    HostOp hA, hB;
    cp_als_opts o;
    cp_status st = residual_setup(h, A, B, f, f_n, hA, hB, o);
    if (st != CP_OK) return st;
    Staged S;
    st = stage_problems(h, 1, &hA, &hB, f_n, f, 1, &o, std::vector<int>(1, 1), S);
    if (st != CP_OK) return st;
    st = ensure_ws(h, S.bytes);
    if (st != CP_OK) return st;
    st = upload_static(h, S, static_cast<char*>(h->ws), nullptr, f, h->stream, false);
    if (st != CP_OK) return st;
    const Problem& pb = S.pk[0].pb;
    st = copy_panels_in(h, h->stream, f_n, pb.V, pb.offV);
    if (st == CP_OK) st = copy_panels_in(h, h->stream, f, pb.U, pb.offU);
    if (st != CP_OK) return st;
    HIP_TRY(launch_residual(S.d_desc, h->stream), "residual launch");
    cp_als_report rep;
    HIP_TRY(hipMemcpyAsync(&rep, pb.reports, sizeof(rep), hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync(report)");
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    *rel_residual = rep.rel_residual;
    return CP_OK;
}

cp_status cp_als_step_adaptive(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                               cp_tensor* f_next, int32_t r_start, double tau, const cp_als_opts* opts,
                               cp_als_report* report, int32_t* final_rank, double* rel_residual) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!f_next || !opts || !report || !final_rank || !rel_residual) return fail(h, CP_ERR_INVALID_ARG, "null argument");
    const int cap = f_next->r;
    if (r_start < 1 || r_start > cap || !(tau >= 0.0)) return fail(h, CP_ERR_INVALID_ARG, "need 1 <= r_start <= cap, tau >= 0");
    cp_als_opts o = *opts;
    o.rank_mode = CP_RANK_ADAPTIVE;
    o.tau_rank = tau;
    o.rank_cap = cap;
    cp_tensor f = *f_next;
    f.r = r_start;
    const cp_status st = cp_als_run(h, A, B, f_n, &f, 1, &o, report, nullptr);
    if (st != CP_OK && st != CP_ERR_NOT_CONVERGED) return st;
    *final_rank = report->final_rank;
    *rel_residual = report->rel_residual;
    return st;
}

cp_status cp_als_run_batched(cp_handle h, int32_t count, const cp_operator* A, const cp_operator* B,
                             const cp_tensor* f_init, cp_tensor* f_io, int32_t n_steps, const cp_als_opts* opts,
                             cp_als_report* reports, double* const* traj) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (count < 1 || !A || !B || !f_init || !f_io || !opts || !reports)
        return fail(h, CP_ERR_INVALID_ARG, "bad batch arguments");
    std::vector<HostOp> hA(count), hB(count);
    for (int i = 0; i < count; ++i) {
        cp_status st = prepare_step(h, &A[i], &B[i], &f_init[i], &f_io[i], n_steps, &opts[i], hA[i], hB[i]);
        if (st != CP_OK) return fail(h, st, "problem " + std::to_string(i) + ": " + h->err);
    }
    return run_problems(h, count, hA.data(), hB.data(), f_init, f_io, n_steps, opts, reports, traj);
}

}  // extern "C"

// A batched launch captured once in a HIP graph: the packed problems live in the plan's own
// device memory, the graph holds the per-run sequence (panels in, barrier counters zeroed,
// the persistent kernel, panels out, reports into pinned host memory) and is replayed on the
// plan's stream (default priority).
struct cp_batch_plan_s {
    Staged S;
    int count = 0, n_steps = 0;
    std::vector<cp_tensor> f_init, f_io;
    hipStream_t stream = nullptr;
    void* dmem = nullptr;
    cp_als_report* rep = nullptr;   // pinned host memory, count * n_steps
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ready = nullptr;
};

namespace {
void plan_release(cp_batch_plan p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ready) (void)hipEventDestroy(p->ready);
    if (p->rep) (void)hipHostFree(p->rep);
    if (p->dmem) (void)hipFree(p->dmem);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}
}  // namespace

extern "C" {

cp_status cp_batch_plan_create(cp_handle h, int32_t count, const cp_operator* A, const cp_operator* B,
                               const cp_tensor* f_init, cp_tensor* f_io, int32_t n_steps, const cp_als_opts* opts,
                               cp_batch_plan* plan) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (count < 1 || !A || !B || !f_init || !f_io || !opts || !plan) return fail(h, CP_ERR_INVALID_ARG, "bad plan arguments");
    *plan = nullptr;
    std::vector<HostOp> hA(count), hB(count);
    for (int i = 0; i < count; ++i) {
        cp_status st = prepare_step(h, &A[i], &B[i], &f_init[i], &f_io[i], n_steps, &opts[i], hA[i], hB[i]);
        if (st != CP_OK) return fail(h, st, "problem " + std::to_string(i) + ": " + h->err);
    }
    cp_batch_plan p = new (std::nothrow) cp_batch_plan_s();
    if (!p) return fail(h, CP_ERR_HIP, "out of host memory");
    p->count = count;
    p->n_steps = n_steps;
    p->f_init.assign(f_init, f_init + count);
    p->f_io.assign(f_io, f_io + count);
    cp_status st = stage_problems(h, count, hA.data(), hB.data(), f_init, f_io, n_steps, opts,
                                  choose_clusters(h, count, hA.data(), hB.data(), f_init, f_io, opts), p->S);
    hipError_t e = hipSuccess;
    const char* what = "";
    if (st == CP_OK) {
        if ((e = hipStreamCreate(&p->stream)) != hipSuccess) what = "hipStreamCreate";
        else if ((e = hipMalloc(&p->dmem, p->S.bytes)) != hipSuccess) what = "hipMalloc";
        else if ((e = hipHostMalloc((void**)&p->rep, (size_t)count * n_steps * sizeof(cp_als_report), hipHostMallocDefault)) != hipSuccess)
            what = "hipHostMalloc";
        else if ((e = hipEventCreateWithFlags(&p->ready, hipEventDisableTiming)) != hipSuccess) what = "hipEventCreate";
        else if ((e = prepare_als()) != hipSuccess) what = "hipFuncSetAttribute";
    }
    if (st == CP_OK && e == hipSuccess)
        st = upload_static(h, p->S, static_cast<char*>(p->dmem), nullptr, f_io, p->stream, true);
    if (st == CP_OK && e == hipSuccess) {
        if ((e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            what = "hipStreamBeginCapture";
        } else {
            st = enqueue_run(h, p->S, p->f_init.data(), p->f_io.data(), p->rep, p->stream, true);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(p->stream, &g);
            p->graph = g;
            if (st == CP_OK && e2 != hipSuccess) {
                e = e2;
                what = "hipStreamEndCapture";
            }
            if (st == CP_OK && e == hipSuccess && (e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess)
                what = "hipGraphInstantiate";
        }
    }
    if (st == CP_OK && e != hipSuccess) st = hip_fail(h, e, what);
    if (st != CP_OK) {
        plan_release(p);
        return st;
    }
    *plan = p;
    return CP_OK;
}

cp_status cp_batch_plan_run(cp_handle h, cp_batch_plan plan, cp_als_report* reports) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!plan || !reports) return fail(h, CP_ERR_INVALID_ARG, "null plan or reports");
    // the run starts after the work already queued on the handle's stream
    HIP_TRY(hipEventRecord(plan->ready, h->stream), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(plan->stream, plan->ready, 0), "hipStreamWaitEvent");
    HIP_TRY(hipGraphLaunch(plan->exec, plan->stream), "hipGraphLaunch");
    HIP_TRY(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
    const int n = plan->count * plan->n_steps;
    std::memcpy(reports, plan->rep, (size_t)n * sizeof(cp_als_report));
    return check_reports(h, reports, n);
}

cp_status cp_batch_plan_destroy(cp_batch_plan plan) {
    if (!plan) return CP_ERR_INVALID_ARG;
    plan_release(plan);
    return CP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// cluster-size tuning
// ---------------------------------------------------------------------------------------
extern "C" {

cp_status cp_tune_cluster(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_n,
                          const cp_tensor* guess, const cp_als_opts* opts, int32_t sweeps, int32_t* best_w,
                          float* best_ms) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!best_w || sweeps < 1) return fail(h, CP_ERR_INVALID_ARG, "best_w is null or sweeps < 1");
    HostOp hA, hB;
    cp_status st = prepare_step(h, A, B, f_n, guess, 1, opts, hA, hB);
    if (st != CP_OK) return st;
    if (with_residual(*opts)) return fail(h, CP_ERR_INVALID_ARG, "problems that form the step residual run on one workgroup");
    cp_als_opts o = *opts;
    o.tol = 0.0;              // every candidate runs the same number of sweeps
    o.max_sweeps = sweeps;
    // a copy of the guess at the start of the workspace, refreshed before every trial (the
    // caller's stays untouched); the trial's packed problem follows it
    size_t nel = 0;
    for (int k = 0; k < guess->d; ++k) nel += (size_t)guess->n[k] * guess->r;
    const size_t gbytes = align_up(nel * 8);
    const int wmax = cluster_size(h, hA, hB, *guess);
    size_t need = 0;
    for (int W = 1; W <= wmax; W *= 2) {
        Staged S;
        st = stage_problems(h, 1, &hA, &hB, f_n, guess, 1, &o, std::vector<int>(1, W), S);
        if (st != CP_OK) return st;
        need = std::max(need, S.bytes);
    }
    st = ensure_ws(h, gbytes + need);
    if (st != CP_OK) return st;
    cp_tensor g = *guess;
    size_t off = 0;
    for (int k = 0; k < g.d; ++k) {
        g.U[k] = reinterpret_cast<double*>(static_cast<char*>(h->ws)) + off;
        g.ld[k] = g.n[k];
        off += (size_t)g.n[k] * g.r;
    }
    char* trial_ws = static_cast<char*>(h->ws) + gbytes;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = 1;
    float tbest = -1.0f;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    for (int W = 1; he == hipSuccess && st == CP_OK && W <= wmax; W *= 2) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && st == CP_OK && he == hipSuccess; ++rep) {   // the first run warms up
            for (int k = 0; k < g.d && he == hipSuccess; ++k)
                he = hipMemcpy2DAsync(g.U[k], (size_t)g.n[k] * 8, guess->U[k], (size_t)guess->ld[k] * 8,
                                      (size_t)g.n[k] * 8, g.r, hipMemcpyDeviceToDevice, h->stream);
            Staged S;
            cp_als_report rp;
            if (he == hipSuccess) st = stage_problems(h, 1, &hA, &hB, f_n, &g, 1, &o, std::vector<int>(1, W), S);
            if (st == CP_OK) st = upload_static(h, S, trial_ws, nullptr, &g, h->stream, false);
            if (st == CP_OK && he == hipSuccess) he = hipEventRecord(e0, h->stream);
            if (st == CP_OK && he == hipSuccess) st = enqueue_run(h, S, f_n, &g, &rp, h->stream);
            if (st == CP_OK && he == hipSuccess) he = hipEventRecord(e1, h->stream);
            if (st == CP_OK && he == hipSuccess) he = hipStreamSynchronize(h->stream);
            if (st == CP_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        }
        if (st == CP_OK && he == hipSuccess && (tbest < 0.0f || ms < tbest)) {
            tbest = ms;
            best = W;
        }
    }
    (void)hipStreamSynchronize(h->stream);   // no copy from a released host buffer may be pending
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != CP_OK) return st;
    if (he != hipSuccess) return hip_fail(h, he, "cluster tuning");
    h->tuned[shape_key(hA, hB, *f_n, *guess, *opts)] = best;
    *best_w = best;
    if (best_ms) *best_ms = tbest;
    return CP_OK;
}

cp_status cp_tune_save(cp_handle h, const char* path) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!path) return fail(h, CP_ERR_INVALID_ARG, "path is null");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(h, CP_ERR_INVALID_ARG, std::string("cannot write ") + path);
    std::fprintf(f, "{\"cluster\": {");
    bool first = true;
    for (const auto& kv : h->tuned) {
        std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    std::fprintf(f, "%s}}\n", first ? "" : "\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? CP_OK : fail(h, CP_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

cp_status cp_tune_load(cp_handle h, const char* path) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!path) return fail(h, CP_ERR_INVALID_ARG, "path is null");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(h, CP_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, got);
    std::fclose(f);
    // {"cluster": {"<key>": <int>, ...}}: keys hold no quotes or escapes
    const size_t c = txt.find("\"cluster\"");
    const size_t o = c == std::string::npos ? c : txt.find('{', c);
    const size_t e = o == std::string::npos ? o : txt.find('}', o);
    if (e == std::string::npos) return fail(h, CP_ERR_INVALID_ARG, std::string("no cluster table in ") + path);
    std::map<std::string, int> add;
    size_t pos = o + 1;
    while (true) {
        const size_t q0 = txt.find('"', pos);
        if (q0 == std::string::npos || q0 > e) break;
        const size_t q1 = txt.find('"', q0 + 1);
        const size_t colon = q1 == std::string::npos ? q1 : txt.find(':', q1);
        if (colon == std::string::npos || colon > e) return fail(h, CP_ERR_INVALID_ARG, "malformed cluster table");
        char* end = nullptr;
        const long v = std::strtol(txt.c_str() + colon + 1, &end, 10);
        if (end == txt.c_str() + colon + 1 || v < 1 || v > 256 || (v & (v - 1)))
            return fail(h, CP_ERR_INVALID_ARG, "bad cluster size in table");
        add[txt.substr(q0 + 1, q1 - q0 - 1)] = (int)v;
        pos = (size_t)(end - txt.c_str());
    }
    for (const auto& kv : add) h->tuned[kv.first] = kv.second;
    return CP_OK;
}

cp_status cp_tune_clear(cp_handle h) {
    if (!h) return CP_ERR_INVALID_ARG;
    h->tuned.clear();
    return CP_OK;
}

// ---------------------------------------------------------------------------------------
// workspace sizes
// ---------------------------------------------------------------------------------------
cp_status cp_workspace_size_step(cp_handle h, const cp_operator* A, const cp_operator* B, const cp_tensor* f_init,
                                 const cp_tensor* source, const cp_tensor* f_io, int32_t n_steps,
                                 const cp_als_opts* opts, size_t* bytes) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!bytes) return fail(h, CP_ERR_INVALID_ARG, "bytes is null");
    cp_status st;
    if (source) {
        cp_tensor g;
        size_t gbytes = 0, goff[CP_MAX_DIMS];
        st = source_tensor(h, B, f_init, source, g, goff, gbytes);
        if (st != CP_OK) return st;
        IdentityOp I(g);
        HostOp hA, hB;
        st = prepare_step(h, A, &I.I, &g, f_io, 1, opts, hA, hB);
        if (st != CP_OK) return st;
        cp_tensor gb = g;
        gb.r = B->n_terms * f_init->r;
        ApplyPlan P;
        st = apply_plan(h, B, f_init, &gb, P);
        if (st != CP_OK) return st;
        size_t rb = 0;
        st = run_bytes(h, 1, &hA, &hB, &g, f_io, 1, opts, &rb);
        if (st != CP_OK) return st;
        *bytes = gbytes + std::max(P.bytes, rb);
        return CP_OK;
    }
    HostOp hA, hB;
    st = prepare_step(h, A, B, f_init, f_io, n_steps, opts, hA, hB);
    if (st != CP_OK) return st;
    size_t need = 0;
    st = run_bytes(h, 1, &hA, &hB, f_init, f_io, n_steps, opts, &need);
    if (st != CP_OK) return st;
    // cp_residual(A, B, f_io, f_init)
    cp_als_opts ro;
    cp_als_default_opts(&ro);
    ro.report_residual = 1;
    Staged S;
    st = stage_problems(h, 1, &hA, &hB, f_init, f_io, 1, &ro, std::vector<int>(1, 1), S);
    if (st != CP_OK) return st;
    need = std::max(need, S.bytes);
    // cp_tune_cluster(A, B, f_init, f_io): a copy of the guess, then each trial
    if (!with_residual(*opts)) {
        cp_als_opts o = *opts;
        o.tol = 0.0;
        size_t nel = 0;
        for (int k = 0; k < f_io->d; ++k) nel += (size_t)f_io->n[k] * f_io->r;
        size_t trial = 0;
        for (int W = 1; W <= cluster_size(h, hA, hB, *f_io); W *= 2) {
            Staged T;
            st = stage_problems(h, 1, &hA, &hB, f_init, f_io, 1, &o, std::vector<int>(1, W), T);
            if (st != CP_OK) return st;
            trial = std::max(trial, T.bytes);
        }
        need = std::max(need, align_up(nel * 8) + trial);
    }
    *bytes = need;
    return CP_OK;
}

cp_status cp_workspace_size_batched(cp_handle h, int32_t count, const cp_operator* A, const cp_operator* B,
                                    const cp_tensor* f_init, const cp_tensor* f_io, int32_t n_steps,
                                    const cp_als_opts* opts, size_t* bytes) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (count < 1 || !A || !B || !f_init || !f_io || !opts || !bytes)
        return fail(h, CP_ERR_INVALID_ARG, "bad batch arguments");
    std::vector<HostOp> hA(count), hB(count);
    for (int i = 0; i < count; ++i) {
        cp_status st = prepare_step(h, &A[i], &B[i], &f_init[i], &f_io[i], n_steps, &opts[i], hA[i], hB[i]);
        if (st != CP_OK) return fail(h, st, "problem " + std::to_string(i) + ": " + h->err);
    }
    return run_bytes(h, count, hA.data(), hB.data(), f_init, f_io, n_steps, opts, bytes);
}

cp_status cp_workspace_size_inner(cp_handle h, const cp_tensor* x, const cp_tensor* y, size_t* bytes) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!bytes) return fail(h, CP_ERR_INVALID_ARG, "bytes is null");
    GramJob job;
    int nch = 0;
    cp_status st = inner_job(h, x, y, job, nch);
    if (st != CP_OK) return st;
    *bytes = inner_bytes(job, nch);
    return CP_OK;
}

cp_status cp_workspace_size_apply(cp_handle h, const cp_operator* L, const cp_tensor* x, size_t* bytes) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!bytes) return fail(h, CP_ERR_INVALID_ARG, "bytes is null");
    ApplyPlan P;
    cp_status st = apply_plan(h, L, x, nullptr, P);
    if (st != CP_OK) return st;
    *bytes = P.bytes;
    return CP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// explicit second-order Adams-Bashforth step (Section 3.2)
// ---------------------------------------------------------------------------------------
namespace {

// A tensor placed in the workspace: element offsets of its panels (column-major n_k x r);
// until bound, the panel pointers name the placeholder.
struct WsTensor {
    cp_tensor t;
    size_t off[CP_MAX_DIMS];
};

// Places a d-dimensional tensor of `cols` columns at byte offset `at`; returns the next
// free (aligned) byte offset.
size_t ws_place(WsTensor& w, int d, const int32_t* n, int cols, size_t at) {
    std::memset(&w.t, 0, sizeof(w.t));
    w.t.d = d;
    w.t.r = cols;
    size_t el = at / 8;
    for (int k = 0; k < d; ++k) {
        w.t.n[k] = n[k];
        w.t.ld[k] = n[k];
        w.t.U[k] = &g_placeholder;
        w.off[k] = el;
        el += (size_t)n[k] * cols;
    }
    return align_up(el * 8);
}

void ws_bind(cp_handle h, WsTensor& w) {
    for (int k = 0; k < w.t.d; ++k) w.t.U[k] = static_cast<double*>(h->ws) + w.off[k];
}

// Columns [c0, c0 + cols) of t.
cp_tensor col_view(const cp_tensor& t, int c0, int cols) {
    cp_tensor v = t;
    v.r = cols;
    for (int k = 0; k < t.d; ++k) v.U[k] = t.U[k] + (size_t)c0 * t.ld[k];
    return v;
}

// alpha times the identity on the grid of t (one term, the coefficient in dimension 0).
struct ScaledIdentity {
    cp_op1d ident[CP_MAX_DIMS];
    double coef;
    int32_t idx[CP_MAX_DIMS] = {0};
    cp_operator op;
    ScaledIdentity(const cp_tensor& t, double alpha) : coef(alpha) {
        std::memset(&op, 0, sizeof(op));
        op.d = t.d;
        op.n_terms = 1;
        op.coef = &coef;
        op.op_index = idx;
        for (int k = 0; k < t.d; ++k) {
            ident[k] = cp_op1d{CP_OP_IDENTITY, t.n[k], 0, nullptr};
            op.n_ops[k] = 1;
            op.ops[k] = &ident[k];
        }
    }
};

cp_status copy_cols(cp_handle h, const cp_tensor& src, cp_tensor& dst, int cols) {
    for (int k = 0; k < src.d; ++k)
        HIP_TRY(hipMemcpy2DAsync(dst.U[k], (size_t)dst.ld[k] * 8, src.U[k], (size_t)src.ld[k] * 8, (size_t)src.n[k] * 8,
                                 cols, hipMemcpyDeviceToDevice, h->stream),
                "hipMemcpy2DAsync(columns)");
    return CP_OK;
}

void skipped_report(cp_als_report* r, int rank) {
    std::memset(r, 0, sizeof(*r));
    r->rel_residual = -1.0;
    r->final_rank = rank;
    r->grown_rank = rank;
}

// Shapes of the three reductions of an AB2 step and the workspace they need.
struct Ab2Plan {
    int d = 0, cap = 0, rp = 0, rc = 0, rw = 0, rw2 = 0, T = 0, tlead = 0, ry = 0, rs = 0;
    bool red1 = false, red2 = false, red3 = false;
    WsTensor W, Wr, Yg, Y, S;
    size_t temps = 0, nested = 0;
};

cp_status ab2_plan(cp_handle h, const cp_operator* L, const cp_tensor* f_prev, const cp_tensor* f_cur,
                   const cp_tensor* f_next, const cp_als_opts* opts, Ab2Plan& P) {
    cp_status st = check_tensor(h, f_prev, "f_prev", CP_MAX_N);
    if (st == CP_OK) st = check_tensor(h, f_cur, "f_cur", CP_MAX_N);
    if (st == CP_OK) st = check_tensor(h, f_next, "f_next", CP_MAX_N);
    if (st == CP_OK) st = check_opts(h, opts);
    if (st != CP_OK) return st;
    if (adaptive(*opts)) return fail(h, CP_ERR_INVALID_ARG, "the AB2 reductions keep a fixed rank cap (rank_mode fixed)");
    const int d = f_cur->d;
    if (f_prev->d != d || f_next->d != d) return fail(h, CP_ERR_SHAPE, "f_prev, f_cur, f_next differ in d");
    for (int k = 0; k < d; ++k)
        if (f_prev->n[k] != f_cur->n[k] || f_next->n[k] != f_cur->n[k])
            return fail(h, CP_ERR_SHAPE, "f_prev, f_cur, f_next differ in n");
    HostOp hL;
    st = check_operator(h, L, "L", d, f_cur->n, false, hL);
    if (st != CP_OK) return st;
    P.d = d;
    P.cap = f_next->r;
    P.rp = f_prev->r;
    P.rc = f_cur->r;
    P.T = L->n_terms;
    P.rw = P.rp + P.rc;
    if (P.rw > CP_MAX_RANK) return fail(h, CP_ERR_SHAPE, "rank(f_prev) + rank(f_cur) exceeds CP_MAX_RANK");
    P.red1 = P.rw > P.cap;
    P.rw2 = std::min(P.rw, P.cap);
    P.red2 = (int64_t)P.T * P.rw2 > P.cap;
    P.tlead = P.red2 ? (P.cap + P.rw2 - 1) / P.rw2 : P.T;
    P.ry = P.red2 ? P.cap : P.T * P.rw2;
    P.rs = P.rc + P.ry;
    if (P.rs > CP_MAX_RANK) return fail(h, CP_ERR_SHAPE, "rank(f_cur) + the reduced rank exceeds CP_MAX_RANK");
    P.red3 = P.rs > P.cap;
    const int32_t* n = f_cur->n;
    size_t off = 0;
    off = ws_place(P.W, d, n, P.rw, off);
    off = ws_place(P.Wr, d, n, P.cap, off);
    off = ws_place(P.Yg, d, n, P.tlead * P.rw2, off);
    off = ws_place(P.Y, d, n, P.ry, off);
    off = ws_place(P.S, d, n, P.rs, off);
    P.temps = off;
    // the nested calls run after the temporaries: the largest of their needs
    size_t need = 0, b = 0;
    ApplyPlan AP;
    st = apply_plan(h, L, f_cur, nullptr, AP);
    if (st != CP_OK) return st;
    need = std::max(need, AP.bytes);
    IdentityOp I(*f_cur);
    HostOp hI, hI2;
    if (P.red1) {
        st = prepare_step(h, &I.I, &I.I, &P.W.t, &P.Wr.t, 1, opts, hI, hI2);
        if (st == CP_OK) st = run_bytes(h, 1, &hI, &hI2, &P.W.t, &P.Wr.t, 1, opts, &b);
        if (st != CP_OK) return st;
        need = std::max(need, b);
    }
    if (P.red2) {
        cp_tensor wv = P.Wr.t;
        wv.r = P.rw2;
        HostOp hA, hB;
        st = prepare_step(h, &I.I, L, &wv, &P.Y.t, 1, opts, hA, hB);
        if (st == CP_OK) st = run_bytes(h, 1, &hA, &hB, &wv, &P.Y.t, 1, opts, &b);
        if (st != CP_OK) return st;
        need = std::max(need, b);
    }
    if (P.red3) {
        cp_tensor fo = *f_next;
        HostOp hA, hB;
        st = prepare_step(h, &I.I, &I.I, &P.S.t, &fo, 1, opts, hA, hB);
        if (st == CP_OK) st = run_bytes(h, 1, &hA, &hB, &P.S.t, &fo, 1, opts, &b);
        if (st != CP_OK) return st;
        need = std::max(need, b);
    }
    P.nested = need;
    return CP_OK;
}

}  // namespace

extern "C" {

cp_status cp_ab2_step(cp_handle h, const cp_operator* L, double dt, const cp_tensor* f_prev, const cp_tensor* f_cur,
                      cp_tensor* f_next, const cp_als_opts* opts, cp_als_report* reports) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!reports || !std::isfinite(dt)) return fail(h, CP_ERR_INVALID_ARG, "reports is null or dt is not finite");
    Ab2Plan P;
    cp_status st = ab2_plan(h, L, f_prev, f_cur, f_next, opts, P);
    if (st != CP_OK) return st;
    st = ensure_ws(h, P.temps + P.nested);
    if (st != CP_OK) return st;
    for (WsTensor* w : {&P.W, &P.Wr, &P.Yg, &P.Y, &P.S}) ws_bind(h, *w);
    const size_t base = P.temps;
    IdentityOp I(*f_cur);
    cp_status worst = CP_OK;
    auto keep = [&](cp_status s) {
        if (s == CP_ERR_NOT_CONVERGED) worst = s;
        return s == CP_OK || s == CP_ERR_NOT_CONVERGED;
    };
    // i) w = 3 f_{n+1} - f_n (the scalars in dimension 0), reduced to rank <= cap
    {
        ScaledIdentity three(*f_cur, 3.0), minus(*f_prev, -1.0);
        cp_tensor a = col_view(P.W.t, 0, P.rc), b = col_view(P.W.t, P.rc, P.rp);
        st = apply_impl(h, &three.op, f_cur, &a, base);
        if (st == CP_OK) st = apply_impl(h, &minus.op, f_prev, &b, base);
        if (st != CP_OK) return st;
    }
    cp_tensor wv = P.W.t;
    if (P.red1) {
        st = copy_cols(h, P.W.t, P.Wr.t, P.cap);   // start: the leading cap columns
        if (st != CP_OK) return st;
        HostOp hA, hB;
        st = prepare_step(h, &I.I, &I.I, &P.W.t, &P.Wr.t, 1, opts, hA, hB);
        if (st == CP_OK) st = run_problems(h, 1, &hA, &hB, &P.W.t, &P.Wr.t, 1, opts, &reports[0], nullptr, base);
        if (!keep(st)) return st;
        wv = P.Wr.t;
    } else {
        skipped_report(&reports[0], P.rw);
    }
    // ii) y = L w, reduced (the ALS fit of L w, from its leading cap columns)
    if (P.red2) {
        cp_operator lead = *L;
        lead.n_terms = P.tlead;
        st = apply_impl(h, &lead, &wv, &P.Yg.t, base);
        if (st == CP_OK) st = copy_cols(h, P.Yg.t, P.Y.t, P.cap);
        if (st != CP_OK) return st;
        HostOp hA, hB;
        st = prepare_step(h, &I.I, L, &wv, &P.Y.t, 1, opts, hA, hB);
        if (st == CP_OK) st = run_problems(h, 1, &hA, &hB, &wv, &P.Y.t, 1, opts, &reports[1], nullptr, base);
        if (!keep(st)) return st;
    } else {
        st = apply_impl(h, L, &wv, &P.Y.t, base);
        if (st != CP_OK) return st;
        skipped_report(&reports[1], P.ry);
    }
    // iii) f_{n+2} = f_{n+1} + (dt / 2) y, reduced
    {
        ScaledIdentity one(*f_cur, 1.0), half(P.Y.t, 0.5 * dt);
        cp_tensor a = col_view(P.S.t, 0, P.rc), b = col_view(P.S.t, P.rc, P.ry);
        st = apply_impl(h, &one.op, f_cur, &a, base);
        if (st == CP_OK) st = apply_impl(h, &half.op, &P.Y.t, &b, base);
        if (st != CP_OK) return st;
    }
    if (P.red3) {
        st = copy_cols(h, P.S.t, *f_next, P.cap);
        if (st != CP_OK) return st;
        HostOp hA, hB;
        st = prepare_step(h, &I.I, &I.I, &P.S.t, f_next, 1, opts, hA, hB);
        if (st == CP_OK) st = run_problems(h, 1, &hA, &hB, &P.S.t, f_next, 1, opts, &reports[2], nullptr, base);
        if (!keep(st)) return st;
    } else {
        st = copy_cols(h, P.S.t, *f_next, P.rs);
        if (st != CP_OK) return st;
        HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        skipped_report(&reports[2], P.rs);
        f_next->r = P.rs;
    }
    return worst != CP_OK ? fail(h, worst, "an AB2 rank reduction reached max_sweeps") : CP_OK;
}

cp_status cp_workspace_size_ab2(cp_handle h, const cp_operator* L, const cp_tensor* f_prev, const cp_tensor* f_cur,
                                const cp_tensor* f_next, const cp_als_opts* opts, size_t* bytes) {
    if (!h) return CP_ERR_INVALID_ARG;
    if (!bytes) return fail(h, CP_ERR_INVALID_ARG, "bytes is null");
    Ab2Plan P;
    cp_status st = ab2_plan(h, L, f_prev, f_cur, f_next, opts, P);
    if (st != CP_OK) return st;
    *bytes = P.temps + P.nested;
    return CP_OK;
}

}  // extern "C"
