// Two-node expansion of linearized factors and device assembly of the
// block-sparse normal equations of a pose graph (GLIM Sec. III-C: a matching
// cost factor between poses T_i and T_j yields H_ii, H_ij, H_jj, b_i, b_j).
//
// A factor's relative pose is T = T_j^-1 T_i (source node i, target node j).
// With right perturbations T_i Exp(xi_i), T_j Exp(xi_j), the relative tangent is
// xi = xi_i - Ad(T^-1) xi_j to first order, so with A = Ad(T^-1):
//   H_ii = H, H_ij = -H A, H_ji = H_ij^T, H_jj = A^T H A, b_i = b, b_j = -A^T b.
//
// Assembly is deterministic: every block of the BSR matrix and every node of
// the right-hand side has a fixed list of contributions (built on the host,
// in factor order), summed in that order in FP64.
#include <algorithm>
#include <map>

#include "vg_device.h"
#include "vg_timeline.h"

struct vg_graph {
    vg_context* ctx = nullptr;
    int64_t N = 0, F = 0, nnzb = 0;
    std::vector<int64_t> row_ptr, col_idx;   // BSR structure (host copy)
    // contributions: per block slot, a list of (factor, kind); kind 0 ii, 1 ij, 2 ji, 3 jj
    int32_t* d_blk_ptr = nullptr;   // nnzb + 1
    int32_t* d_blk_item = nullptr;  // packed (factor << 2 | kind)
    int32_t* d_rhs_ptr = nullptr;   // N + 1
    int32_t* d_rhs_item = nullptr;  // packed (factor << 1 | side), side 0 = i, 1 = j
    double* d_adj = nullptr;        // F x 36: Ad(T^-1) per factor
    uint32_t magic = 0;
};

namespace vg {

// Ad(T^-1) for T = (R, t): T^-1 = (R^T, -R^T t) and Ad(R', t') = [[R', 0], [(t')x R', R']].
__global__ void k_graph_adjoint(int64_t F, const double* __restrict__ poses, double* __restrict__ adj) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* P = poses + 12 * f;
    double Rt[9], tp[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Rt[3 * i + j] = P[3 * j + i];
    for (int i = 0; i < 3; ++i) tp[i] = -(Rt[3 * i] * P[9] + Rt[3 * i + 1] * P[10] + Rt[3 * i + 2] * P[11]);
    const double tx[9] = {0, -tp[2], tp[1], tp[2], 0, -tp[0], -tp[1], tp[0], 0};
    double* A = adj + 36 * f;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) A[6 * i + j] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[6 * i + j] = Rt[3 * i + j];
            A[6 * (3 + i) + 3 + j] = Rt[3 * i + j];
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += tx[3 * i + q] * Rt[3 * q + j];
            A[6 * (3 + i) + j] = s;
        }
}

// One 64-thread block per BSR block; thread k < 36 owns entry (r, c) = (k / 6, k % 6).
__global__ void k_graph_blocks(const int32_t* __restrict__ blk_ptr, const int32_t* __restrict__ blk_item,
                               const double* __restrict__ lin, const double* __restrict__ adj,
                               double* __restrict__ values) {
    const int64_t s = blockIdx.x;
    const int k = threadIdx.x;
    if (k >= 36) return;
    const int r = k / 6, c = k % 6;
    double acc = 0.0;
    for (int32_t it = blk_ptr[s]; it < blk_ptr[s + 1]; ++it) {
        const int32_t item = blk_item[it];
        const int64_t f = item >> 2;
        const int kind = item & 3;
        const double* H = lin + (int64_t)kOutRow * f + 1;
        const double* A = adj + 36 * f;
        double v = 0.0;
        if (kind == 0) {
            v = H[6 * r + c];
        } else if (kind == 1) {   // -(H A)_{rc}
            for (int q = 0; q < 6; ++q) v -= H[6 * r + q] * A[6 * q + c];
        } else if (kind == 2) {   // (H_ij)^T_{rc} = -(H A)_{cr}
            for (int q = 0; q < 6; ++q) v -= H[6 * c + q] * A[6 * q + r];
        } else {                  // (A^T H A)_{rc}
            for (int p = 0; p < 6; ++p) {
                double hq = 0.0;
                for (int q = 0; q < 6; ++q) hq += H[6 * p + q] * A[6 * q + c];
                v += A[6 * p + r] * hq;
            }
        }
        acc += v;
    }
    values[36 * s + k] = acc;
}

// One 64-thread block per node; thread r < 6 owns rhs entry r; thread 6 sums e.
__global__ void k_graph_rhs(const int32_t* __restrict__ rhs_ptr, const int32_t* __restrict__ rhs_item,
                            const double* __restrict__ lin, const double* __restrict__ adj, double* __restrict__ rhs) {
    const int64_t node = blockIdx.x;
    const int r = threadIdx.x;
    if (r >= 6) return;
    double acc = 0.0;
    for (int32_t it = rhs_ptr[node]; it < rhs_ptr[node + 1]; ++it) {
        const int32_t item = rhs_item[it];
        const int64_t f = item >> 1;
        const double* b = lin + (int64_t)kOutRow * f + 37;
        if ((item & 1) == 0) {
            acc += b[r];
        } else {                   // -(A^T b)_r
            const double* A = adj + 36 * f;
            double v = 0.0;
            for (int q = 0; q < 6; ++q) v += A[6 * q + r] * b[q];
            acc -= v;
        }
    }
    rhs[6 * node + r] = acc;
}

}  // namespace vg

using namespace vg;

namespace {
constexpr uint32_t kGraphMagic = 0x62A90001u;
bool graph_ok(const vg_graph* g) { return g != nullptr && g->magic == kGraphMagic; }
vg_status g_invalid(const char* m) {
    set_error(m);
    return VG_ERR_INVALID_ARG;
}
void graph_free(vg_graph* g) {
    if (g->d_blk_ptr) (void)hipFree(g->d_blk_ptr);
    if (g->d_blk_item) (void)hipFree(g->d_blk_item);
    if (g->d_rhs_ptr) (void)hipFree(g->d_rhs_ptr);
    if (g->d_rhs_item) (void)hipFree(g->d_rhs_item);
    if (g->d_adj) (void)hipFree(g->d_adj);
}
template <typename T>
hipError_t up(T** d, const std::vector<T>& h) {
    hipError_t e = hipMalloc((void**)d, sizeof(T) * std::max<size_t>(h.size(), 1));
    if (e == hipSuccess && !h.empty()) e = hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
    return e;
}
}  // namespace

extern "C" vg_status vg_create_graph(vg_context* ctx, int64_t N, int64_t F, const int64_t* node_i,
                                     const int64_t* node_j, vg_graph** out) {
    set_error("");
    if (!context_ok(ctx)) {
        set_error("invalid context");
        return VG_ERR_STATE;
    }
    if (out == nullptr) return g_invalid("out is NULL");
    *out = nullptr;
    if (N < 1 || F < 0 || N >= (1ll << 30) || F >= (1ll << 29)) return g_invalid("N or F out of range");
    if (F > 0 && (node_i == nullptr || node_j == nullptr)) return g_invalid("node arrays are NULL");
    for (int64_t f = 0; f < F; ++f)
        if (node_i[f] < 0 || node_i[f] >= N || node_j[f] < 0 || node_j[f] >= N || node_i[f] == node_j[f])
            return g_invalid("factor nodes must be distinct and in [0, N)");
    // blocks: (r, c) -> ordered contribution list
    std::map<std::pair<int64_t, int64_t>, std::vector<int32_t>> blocks;
    std::vector<std::vector<int32_t>> rhs((size_t)N);
    for (int64_t f = 0; f < F; ++f) {
        const int64_t i = node_i[f], j = node_j[f];
        blocks[{i, i}].push_back((int32_t)(f << 2 | 0));
        blocks[{i, j}].push_back((int32_t)(f << 2 | 1));
        blocks[{j, i}].push_back((int32_t)(f << 2 | 2));
        blocks[{j, j}].push_back((int32_t)(f << 2 | 3));
        rhs[i].push_back((int32_t)(f << 1 | 0));
        rhs[j].push_back((int32_t)(f << 1 | 1));
    }
    for (int64_t n = 0; n < N; ++n) blocks[{n, n}];   // every node has a diagonal block
    auto* g = new vg_graph();
    g->ctx = ctx;
    g->N = N;
    g->F = F;
    g->row_ptr.assign(N + 1, 0);
    std::vector<int32_t> bptr, bitem, rptr, ritem;
    bptr.push_back(0);
    for (auto& kv : blocks) {
        g->row_ptr[kv.first.first + 1] += 1;
        g->col_idx.push_back(kv.first.second);
        for (int32_t it : kv.second) bitem.push_back(it);
        bptr.push_back((int32_t)bitem.size());
    }
    for (int64_t n = 0; n < N; ++n) g->row_ptr[n + 1] += g->row_ptr[n];
    g->nnzb = (int64_t)g->col_idx.size();
    rptr.push_back(0);
    for (int64_t n = 0; n < N; ++n) {
        for (int32_t it : rhs[n]) ritem.push_back(it);
        rptr.push_back((int32_t)ritem.size());
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = up(&g->d_blk_ptr, bptr);
    if (e == hipSuccess) e = up(&g->d_blk_item, bitem);
    if (e == hipSuccess) e = up(&g->d_rhs_ptr, rptr);
    if (e == hipSuccess) e = up(&g->d_rhs_item, ritem);
    if (e == hipSuccess) e = hipMalloc(&g->d_adj, sizeof(double) * 36 * std::max<int64_t>(F, 1));
    if (e != hipSuccess) {
        graph_free(g);
        delete g;
        return hip_fail(e, "graph upload");
    }
    g->magic = kGraphMagic;
    *out = g;
    return VG_OK;
}

extern "C" vg_status vg_graph_structure(const vg_graph* g, int64_t* nnz_blocks, int64_t* row_ptr, int64_t* col_idx) {
    set_error("");
    if (!graph_ok(g)) {
        set_error("invalid graph");
        return VG_ERR_STATE;
    }
    if (nnz_blocks) *nnz_blocks = g->nnzb;
    if (row_ptr) std::copy(g->row_ptr.begin(), g->row_ptr.end(), row_ptr);
    if (col_idx) std::copy(g->col_idx.begin(), g->col_idx.end(), col_idx);
    return VG_OK;
}

extern "C" vg_status vg_graph_assemble_async(vg_graph* g, const double* d_poses, const double* d_lin,
                                             double* d_values, double* d_rhs) {
    const vg::TimelineRange range_("vg_graph_assemble_async");
    set_error("");
    if (!graph_ok(g)) {
        set_error("invalid graph");
        return VG_ERR_STATE;
    }
    if ((g->F > 0 && (d_poses == nullptr || d_lin == nullptr)) || d_values == nullptr || d_rhs == nullptr)
        return g_invalid("NULL device pointer");
    VG_HIP(hipSetDevice(g->ctx->device));
    hipStream_t st = g->ctx->stream;
    if (g->F > 0) {
        k_graph_adjoint<<<(int)((g->F + 63) / 64), 64, 0, st>>>(g->F, d_poses, g->d_adj);
        VG_HIP(hipGetLastError());
    }
    k_graph_blocks<<<(int)g->nnzb, 64, 0, st>>>(g->d_blk_ptr, g->d_blk_item, d_lin, g->d_adj, d_values);
    VG_HIP(hipGetLastError());
    k_graph_rhs<<<(int)g->N, 64, 0, st>>>(g->d_rhs_ptr, g->d_rhs_item, d_lin, g->d_adj, d_rhs);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

extern "C" vg_status vg_graph_destroy(vg_graph* g) {
    set_error("");
    if (!graph_ok(g)) {
        set_error("invalid graph");
        return VG_ERR_STATE;
    }
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    graph_free(g);
    g->magic = 0;
    delete g;
    return VG_OK;
}
