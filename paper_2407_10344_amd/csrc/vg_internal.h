// Internal declarations of the VGICP device library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vgicp.h"

namespace vg {

// ---------------------------------------------------------------- constants

constexpr int kMaxLevels = 4;
constexpr int kChunk = 64;              // points per anchor chunk == one wavefront
constexpr int kKeyBits = 14;            // bits per axis of a packed relative voxel key
constexpr int kKeyBias = 1 << (kKeyBits - 1);   // relative keys live in [-8192, 8191]
constexpr int kBlockShift = 2;          // voxel blocks of 4 x 4 x 4
constexpr int kBlockBits = kKeyBits - kBlockShift;   // 12 bits per axis of a block key
constexpr int kBaseBits = 28;           // first-record index bits of a block entry
constexpr uint64_t kBaseMask = (1ull << kBaseBits) - 1;
// voxels per level: records are addressed by 32-bit byte offsets (64 B each), so
// fewer than 2^26; this also keeps a valid entry word from ever being all ones
constexpr int64_t kMaxVoxels = ((int64_t)1 << 26) - 1;
constexpr uint64_t kEmpty = ~0ull;      // empty block-table entry
constexpr int kTerms = 28;              // e, 21 upper-triangular H, 6 b
// partial row of a tile (FP64): 28 terms, inliers per level, then the work the
// tile did: source points walked (chunks not culled), table lookups per level
// (point-levels inside the level's key box), chunks walked
constexpr int kRowInl = kTerms;                  // 4: points with a voxel, per level
constexpr int kRowWalk = kRowInl + 4;            // 1: source points walked
constexpr int kRowProbe = kRowWalk + 1;          // 4: table lookups, per level
constexpr int kRowChunks = kRowProbe + 4;        // 1: chunks walked
constexpr int kRow = 40;
constexpr int kWork = 8;                // per-factor work counts: walked points, walked chunks, lookups (4), 0, 0
constexpr int kMaxTileChunks = 128;     // chunks whose data a tile holds in LDS at once
constexpr int kMaxTilePoints = 32768;   // points per tile (taken in batches of kMaxTileChunks chunks)
constexpr int kRec32 = 16;              // floats per compensated voxel record (64 B: 4 FP32 + 6 FP64)
constexpr int kRecN = 12;               // floats per absolute-FP32 voxel record
constexpr int kRec64 = 10;              // doubles per FP64 voxel record
constexpr int kOutRow = 43;             // e, H (36), b (6)
constexpr int kParts = 8;               // tile partitions = XCDs of an MI355X

enum Mode { kLin = 0, kEval = 1, kBwd = 2, kCount = 3 };
enum Prec { kN32 = VG_FP32, kC32 = VG_FP32_COMPENSATED, kF64 = VG_FP64 };

// ---------------------------------------------------------------- device descriptors

// One level of a target voxel map as the kernels see it.
struct LevelDesc {
    const uint64_t* slots;   // 2^log2cap block entries of two words:
                             //   [(36-bit block key << 28) | first record, 64-bit occupancy]
    const float* rec32;      // V x 16 floats (64 B): mean - voxel centre (3 FP32), count (FP32), cov (6 FP64)
    const float* recN;       // V x 12: FP32 absolute mean (3), cov (6), pad
    const double* rec64;     // V x 10: absolute mean (3), cov (6), pad
    uint32_t log2cap;
    int32_t scale;           // r_coarsest / r_l (power of two)
    int32_t log2scale;       // log2 of scale
    float r, inv_r;
    double r64, inv_r64;
    int64_t K0[3];           // absolute key of the map origin at this level
    int32_t kmin[3], kmax[3];// bounding box of the level's relative keys (empty: min > max)
    int32_t kbox0[3];        // the same box as kbox0 + [0, kboxw] (empty level: the single key 0)
    uint32_t kboxw[3];
    double blo[3], bhi[3];   // the same box in metres, target frame (empty level: blo > bhi)
};

// One factor: a source cloud (internal Morton order) matched into a target map.
struct FactorDesc {
    const float* dxyz;       // 3 x n_pad SoA offsets from the chunk anchor
    const float* cov;        // 6 x n_pad SoA covariances
    const float* nrm;        // 3 x n_pad SoA normals or nullptr
    const double* anchor;    // n_chunks x 3 absolute anchors (source frame)
    const float* cbound;     // n_chunks x 8: chunk bounds around the anchor (m): box centre offset (3),
                             //   ball radius, box half extents (3), 0
    const float* axyz;       // 3 x n_pad absolute FP32 positions
    const double* xyz64;     // 3 x n_pad absolute FP64 positions
    const double* cov64;     // 6 x n_pad FP64 covariances
    const double* nrm64;     // 3 x n_pad FP64 normals or nullptr
    const int32_t* perm;     // internal index -> caller index
    int64_t n, n_pad;
    int64_t grad_offset;     // first row of this source in the concatenated point gradient
    int64_t grad_slab;       // -1 if no other factor of the batch uses this source; otherwise the
                             //   first row of this factor's own rows in the per-factor gradient
                             //   buffer, summed per source in factor order afterwards
    int32_t L;
    int32_t pad_;
    double src_origin[3];    // o_s: the re-centring origin of the source
    double viewpoint[3];     // target viewpoint (target frame) for surface validation
    LevelDesc lv[kMaxLevels];
};

// A source used by several factors of a batch: its rows of the point gradient
// are the sum, in factor order, of those factors' rows in the per-factor buffer.
struct SharedSrc {
    int64_t row0;            // first of its rows among all shared sources' rows
    int64_t n;               // points
    int64_t grad_offset;     // first row in the concatenated point gradient
    int32_t f0, f1;          // its factors' entries [f0, f1) in the slab-offset list
};

// Device buffers one launch of the tile kernel and reduction works in.
struct Workspace {
    double* partials;        // n_tiles x kRow
    uint32_t* counter;       // kParts tile counters (zero before the first launch)
    float* posef;            // F x 16 staged FP32 poses
    int64_t* work;           // F x kWork work counts, or nullptr
};

struct Tile {
    int32_t factor;
    int32_t chunk0;          // first chunk of the factor's source
    int32_t nchunks;
    int32_t pad;
};

// ---------------------------------------------------------------- host objects

struct Level {
    double r = 0;
    int64_t K0[3] = {0, 0, 0};
    int64_t V = 0;
    uint32_t log2cap = 0;      // block-table entries = 2^log2cap
    int64_t n_blocks = 0;
    uint64_t* slots = nullptr; // 2 words per entry
    float* rec32 = nullptr;
    float* recN = nullptr;
    double* rec64 = nullptr;
    uint64_t* keys = nullptr;   // V packed relative keys, ascending (canonical order)
    int32_t* counts = nullptr;  // V, canonical order
    int32_t* lex2rec = nullptr; // V: canonical index -> record index (records are block ordered)
    int32_t kmin[3] = {1, 1, 1}, kmax[3] = {0, 0, 0};   // relative key bounding box
};

}  // namespace vg

struct vg_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* ws = nullptr;          // grow-only device workspace of the preprocessing calls
    size_t ws_bytes = 0;
    int num_cu = 0;
    void* scratch = nullptr;     // this device's fixed scratch array (device address), or nullptr
    std::string arch;
    std::string name;
    uint32_t magic = 0;
};

struct vg_voxelmap {
    vg_context* ctx = nullptr;
    int L = 0;
    double origin[3] = {0, 0, 0};
    vg::Level lv[vg::kMaxLevels];
    int users = 0;
    uint32_t magic = 0;
};

struct vg_source {
    vg_context* ctx = nullptr;
    int64_t n = 0, n_pad = 0, n_chunks = 0;
    double origin[3] = {0, 0, 0};
    bool has_normals = false;
    float* dxyz = nullptr;
    float* cov = nullptr;
    float* nrm = nullptr;
    double* anchor = nullptr;
    float* cbound = nullptr;   // per chunk: box centre offset (3), ball radius, box half extents (3), 0 (m)
    float* axyz = nullptr;
    double* xyz64 = nullptr;
    double* cov64 = nullptr;
    double* nrm64 = nullptr;
    int32_t* perm = nullptr;   // internal -> caller
    double extent = 0.0;       // upper bound of |mu - origin| over its points (m), from the chunk bounds
    int users = 0;
    uint32_t magic = 0;
};

// A preprocessed frame (downsampled points, neighbours, covariances, normals).
struct vg_cloud {
    vg_context* ctx = nullptr;
    int64_t m = 0;              // downsampled points
    int32_t k = 0;              // neighbours per point
    double* xyz = nullptr;      // m x 3
    double* cov = nullptr;      // m x 6 regularised
    double* cov_raw = nullptr;  // m x 6 neighbour covariance
    double* nrm = nullptr;      // m x 3
    int32_t* counts = nullptr;  // m input points per voxel
    int32_t* nbr = nullptr;     // m x k
    double* d2 = nullptr;       // m x k
    void* block = nullptr;      // one allocation holding every array above
    double first[3] = {0, 0, 0};// host copy of point 0 (origins of sources / maps made from the cloud)
    uint32_t magic = 0;
};

struct vg_batch {
    vg_context* ctx = nullptr;
    int64_t F = 0;
    int L = 0;
    vg_batch_options opt{};
    std::vector<vg_source*> src;
    std::vector<vg_voxelmap*> tgt;
    std::vector<vg::FactorDesc> h_fac;
    std::vector<vg::Tile> h_tiles;
    std::vector<int32_t> h_tile_first;   // F + 1
    std::vector<int64_t> grad_offsets;   // per unique source
    int64_t total_points = 0;
    int64_t grad_rows = 0;               // rows of the concatenated point gradient
    int block = 256, tile_points = 2048, grid = 0, blocks_per_cu = 0;
    int tile_order = 1;                  // 1 contiguous per XCD, 2 round-robin over XCDs
    // device buffers
    vg::FactorDesc* d_fac = nullptr;
    vg::Tile* d_tiles = nullptr;
    int32_t* d_tile_first = nullptr;
    double* d_partials = nullptr;
    uint32_t* d_counter = nullptr;
    double* d_poses = nullptr;
    float* d_posef = nullptr;       // F x 16 staged FP32 poses
    double* d_out = nullptr;        // F x 43
    int64_t* d_inliers = nullptr;   // F x L
    int64_t* d_work = nullptr;      // F x kWork work counts of the last linearize / evaluate / overlap
    double* d_e = nullptr;          // F (evaluate)
    double* d_lm = nullptr;         // LM scratch
    // sources shared by several factors (deterministic point gradients)
    std::vector<vg::SharedSrc> h_shared;
    std::vector<int64_t> h_slab_off;     // per shared source, its factors' slab rows, factor order
    int64_t slab_rows = 0;
    int64_t shared_rows = 0;
    vg::SharedSrc* d_shared = nullptr;
    int64_t* d_slab_off = nullptr;
    void* d_gslab = nullptr;             // per-factor point gradients (grown on first use)
    size_t gslab_bytes = 0;
    double max_source_extent = 0.0;      // largest |mu - o_s| over the batch's sources (m)
    // pinned host staging (one upload, one download)
    double* h_poses = nullptr;
    double* h_out = nullptr;
    int64_t* h_inliers = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t magic = 0;
};

namespace vg {

// ---------------------------------------------------------------- error state

void set_error(const std::string& msg);
bool context_ok(const vg_context* c);
vg_status hip_fail(hipError_t e, const char* what);

#define VG_HIP(call)                                        \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return vg::hip_fail(_e, #call);\
    } while (0)

// ---------------------------------------------------------------- launchers (device code)

vg_status build_level(vg_context* ctx, const double* d_xyz, const double* d_cov, int64_t n, double r,
                      const double origin[3], Level* out);
vg_status export_level(vg_context* ctx, const Level& lv, int64_t* keys, double* means, double* covs,
                       int64_t* counts);
void free_level(Level* lv);

// frame preprocessing: d_xyz n x 3 FP64 device input; fills every array of *out
vg_status preprocess_frame(vg_context* ctx, const double* d_xyz, int64_t n, double r, int k, const double sensor[3],
                           vg_cloud* out);
void free_cloud(vg_cloud* c);

vg_status layout_source(vg_context* ctx, vg_source* s, const double* d_xyz, const double* d_cov,
                        const double* d_nrm);
vg_status set_source_points(vg_context* ctx, vg_source* s, const void* d_xyz, int dtype);

// launch the tile kernel over tiles [t0, t1) and the reduction over factors [f0, f1)
// f0, f1: the factors those tiles belong to (their poses are staged to FP32 first)
// ws: the buffers of the launch (the batch's own, or a caller-provided scratch)
vg_status launch_tiles(vg_batch* b, const Workspace& ws, int mode, const double* d_poses, int32_t t0, int32_t t1,
                       int grid, const double* d_grad_e, void* d_grad_points, int points_dtype, int64_t f0,
                       int64_t f1);
vg_status launch_reduce(vg_batch* b, const Workspace& ws, int mode, const double* d_poses, int32_t f0, int32_t f1,
                        double* d_out, int64_t* d_inliers, const double* d_grad_e, const double* d_jr,
                        double* d_grad_xi);
// rows of shared sources: sum of their factors' per-factor rows in factor order
vg_status launch_grad_combine(vg_batch* b, void* d_grad_points, int points_dtype);
vg_status launch_correspondences(vg_batch* b, const double* d_pose, int64_t factor, int64_t* d_keys,
                                 int32_t* d_found);
vg_status launch_zero(vg_context* ctx, void* d_ptr, size_t bytes);
vg_status launch_se3_retract(vg_context* ctx, int64_t F, const double* d_T0, const double* d_xi, double* d_T,
                             double* d_jr);
// LM on the device: propose solves (H + lambda diag H) delta = -b from the
// linearization rows d_out and writes T Exp(delta) to d_cand (d_valid = 0 and
// d_cand = T where the damped matrix is not SPD); accept keeps the candidate
// iff it is valid and e decreases (lambda / 10), else keeps T (lambda x 10),
// writing e at T and the decision to d_e / d_accepted at column `col` of rows
// of length `stride` (either may be nullptr).
vg_status launch_lm_propose(vg_batch* b, const double* d_out, const double* d_lambda, const double* d_poses,
                            double* d_cand, int32_t* d_valid);
vg_status launch_lm_accept(vg_batch* b, const double* d_out, const double* d_e_new, double* d_lambda,
                           double* d_poses, const double* d_cand, const int32_t* d_valid, double* d_e,
                           int32_t* d_accepted, int32_t stride, int32_t col);
vg_status launch_fill(vg_context* ctx, double* d_ptr, int64_t n, double v);

}  // namespace vg
