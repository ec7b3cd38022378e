// C ABI of the VGICP library: validation, handle lifetime, batch scheduling
// (tile list, plain per-factor loop, batched launch, captured hipGraph),
// Levenberg-Marquardt driver and the launch-shape autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "vg_internal.h"
#include "vg_timeline.h"

// Device scratch of the allocation-free linearization (vg_linearize_noalloc):
// tile counters, staged FP32 poses and tile partial rows.  Every device the
// library runs on holds its own copy until the process ends; host code reaches
// it only through the per-device address taken with hipGetSymbolAddress.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr uint32_t kCtxMagic = 0xC0FFEE01u;
constexpr uint32_t kMapMagic = 0x3A900001u;
constexpr uint32_t kSrcMagic = 0x50CE0001u;
constexpr uint32_t kBatMagic = 0xBA7C0001u;

// Largest distance (m) of a source point from its re-centring origin that the
// compensated FP32 mode accepts: its per-point lever arms are FP32, and the
// rotational part of b cancels across the cloud, so the relative error of b
// grows with the extent (below 1e-6 for clouds of a few hundred metres, ~3e-4
// for one spanning 4 km).
constexpr double kMaxCompensatedExtent = 500.0;

thread_local std::string g_err;

// Device address of `scratch` on each device, taken once per device when the
// first context on it is created.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

bool finite_all(const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Leading principal minors of [a b c; b d e; c e f] all positive.
bool spd6(const double* c) {
    const double a = c[0], b = c[1], cc = c[2], d = c[3], e = c[4], f = c[5];
    if (!(a > 0.0)) return false;
    const double m2 = a * d - b * b;
    if (!(m2 > 0.0)) return false;
    const double det = a * (d * f - e * e) - b * (b * f - cc * e) + cc * (b * e - cc * d);
    return det > 0.0;
}

bool is_pow2(double r) {
    int ex = 0;
    const double m = std::frexp(r, &ex);
    return m == 0.5;
}

vg_status invalid(const std::string& msg) {
    vg::set_error(msg);
    return VG_ERR_INVALID_ARG;
}

vg_status state_err(const std::string& msg) {
    vg::set_error(msg);
    return VG_ERR_STATE;
}

bool ctx_ok(const vg_context* c) { return c != nullptr && c->magic == kCtxMagic; }
bool map_ok(const vg_voxelmap* m) { return m != nullptr && m->magic == kMapMagic; }
bool src_ok(const vg_source* s) { return s != nullptr && s->magic == kSrcMagic; }
bool bat_ok(const vg_batch* b) { return b != nullptr && b->magic == kBatMagic; }

// Poses: finite, R orthonormal to 1e-6, det(R) > 0.
vg_status check_poses(const double* poses, int64_t F) {
    if (poses == nullptr) return invalid("poses is NULL");
    for (int64_t f = 0; f < F; ++f) {
        const double* p = poses + 12 * f;
        if (!finite_all(p, 12)) return invalid("pose " + std::to_string(f) + " is not finite");
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += p[3 * k + i] * p[3 * k + j];
                if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-6)
                    return invalid("pose " + std::to_string(f) + " rotation is not orthonormal");
            }
        const double det = p[0] * (p[4] * p[8] - p[5] * p[7]) - p[1] * (p[3] * p[8] - p[5] * p[6]) +
                           p[2] * (p[3] * p[7] - p[4] * p[6]);
        if (det <= 0.0) return invalid("pose " + std::to_string(f) + " rotation has det <= 0");
    }
    return VG_OK;
}

template <typename T>
vg_status dev_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        vg::set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return VG_ERR_OOM;
    }
    return VG_OK;
}

template <typename T>
vg_status host_alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipHostMalloc((void**)p, sizeof(T) * count, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        vg::set_error(std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
        return VG_ERR_OOM;
    }
    return VG_OK;
}

#define VG_TRY(x)                          \
    do {                                   \
        vg_status _s = (x);                \
        if (_s != VG_OK) return _s;        \
    } while (0)

void dfree(void* p) {
    if (p) (void)hipFree(p);
}
void hfree(void* p) {
    if (p) (void)hipHostFree(p);
}

}  // namespace

namespace vg {

void set_error(const std::string& msg) { g_err = msg; }
bool context_ok(const vg_context* c) { return ctx_ok(c); }

vg_status hip_fail(hipError_t e, const char* what) {
    (void)hipGetLastError();
    g_err = std::string("HIP error in ") + what + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VG_ERR_OOM : VG_ERR_HIP;
}

}  // namespace vg

using namespace vg;

// ============================================================================ context

extern "C" const char* vg_last_error(void) { return g_err.c_str(); }

extern "C" int32_t vg_version(void) { return 10000; }

extern "C" vg_status vg_context_create(int32_t device, void* hip_stream, vg_context** out) {
    g_err.clear();
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        (void)hipGetLastError();
        set_error(std::string("no HIP device available") + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : ""));
        return VG_ERR_HIP;
    }
    if (device < 0 || device >= count) return invalid("device index out of range");
    VG_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    VG_HIP(hipGetDeviceProperties(&prop, device));
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0) {
        set_error("device " + std::to_string(device) + " is " + arch + "; this library is built for gfx950 only");
        return VG_ERR_HIP;
    }
    auto* c = new vg_context();
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    if (device < kMaxDevices) {
        // this device's copy of the fixed scratch (device current); a failure only
        // disables vg_linearize_noalloc, which reports it
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_done[device]) {
            void* ptr = nullptr;
            const hipError_t se = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (se != hipSuccess) (void)hipGetLastError();
            g_scratch_err[device] = se;
            g_scratch_ptr[device] = se == hipSuccess ? ptr : nullptr;
            g_scratch_done[device] = true;
        }
        c->scratch = g_scratch_ptr[device];
    }
    c->arch = arch;
    c->name = prop.name;
    if (hip_stream != nullptr) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
        c->own_stream = true;
    }
    c->magic = kCtxMagic;
    *out = c;
    return VG_OK;
}

extern "C" vg_status vg_context_destroy(vg_context* ctx) {
    g_err.clear();
    if (!ctx_ok(ctx)) return state_err("invalid context");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->magic = 0;
    delete ctx;
    return VG_OK;
}

// ============================================================================ voxel maps

// Voxel map from device FP64 arrays; first = host copy of point 0 (the origin).
static vg_status make_voxelmap(vg_context* ctx, const double* d_xyz, const double* d_cov, int64_t n,
                               const double* resolutions, int32_t L, const double* first, vg_voxelmap** out) {
    auto* m = new vg_voxelmap();
    m->ctx = ctx;
    m->L = L;
    const double rmax = resolutions[L - 1];
    for (int a = 0; a < 3; ++a) m->origin[a] = (n > 0) ? rmax * std::nearbyint(first[a] / rmax) : 0.0;
    vg_status st = VG_OK;
    for (int l = 0; l < L && st == VG_OK; ++l)
        st = build_level(ctx, d_xyz, d_cov, n, resolutions[l], m->origin, &m->lv[l]);
    if (st != VG_OK) {
        for (int l = 0; l < kMaxLevels; ++l) free_level(&m->lv[l]);
        delete m;
        return st;
    }
    m->magic = kMapMagic;
    *out = m;
    return VG_OK;
}

static vg_status check_resolutions(const double* resolutions, int32_t L) {
    if (L < 1 || L > kMaxLevels) return invalid("L must be in 1..4");
    if (resolutions == nullptr) return invalid("resolutions is NULL");
    for (int l = 0; l < L; ++l) {
        const double r = resolutions[l];
        if (!(std::isfinite(r) && r > 0.0 && is_pow2(r))) return invalid("each resolution must be a positive power of two");
        if (l > 0 && !(r > resolutions[l - 1])) return invalid("resolutions must be strictly ascending");
    }
    return VG_OK;
}

extern "C" vg_status vg_build_voxelmap(vg_context* ctx, const double* xyz, const double* cov, int64_t n,
                                       const double* resolutions, int32_t L, vg_voxelmap** out) {
    g_err.clear();
    const TimelineRange range_("vg_build_voxelmap");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    if (n < 0) return invalid("n < 0");
    if (n > 0 && (xyz == nullptr || cov == nullptr)) return invalid("xyz or cov is NULL");
    if (n >= (int64_t)1 << 31) return invalid("n must be below 2^31");
    VG_TRY(check_resolutions(resolutions, L));
    if (n > 0 && !finite_all(xyz, 3 * n)) return invalid("xyz has non-finite values");
    if (n > 0 && !finite_all(cov, 6 * n)) return invalid("cov has non-finite values");
    for (int64_t i = 0; i < n; ++i)
        if (!spd6(cov + 6 * i)) {
            set_error("covariance of point " + std::to_string(i) + " is not SPD");
            return VG_ERR_NOT_SPD;
        }
    VG_HIP(hipSetDevice(ctx->device));
    double *d_xyz = nullptr, *d_cov = nullptr;
    vg_status st = VG_OK;
    do {
        if ((st = dev_alloc(&d_xyz, 3 * n)) != VG_OK) break;
        if ((st = dev_alloc(&d_cov, 6 * n)) != VG_OK) break;
        hipError_t e = hipSuccess;
        if (n > 0) {
            e = hipMemcpyAsync(d_xyz, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_cov, cov, sizeof(double) * 6 * n, hipMemcpyHostToDevice, ctx->stream);
        }
        if (e != hipSuccess) {
            st = hip_fail(e, "voxelmap upload");
            break;
        }
        st = make_voxelmap(ctx, d_xyz, d_cov, n, resolutions, L, xyz, out);
    } while (0);
    dfree(d_xyz);
    dfree(d_cov);
    return st;
}

extern "C" vg_status vg_voxelmap_info(const vg_voxelmap* map, int32_t level, int64_t* n_voxels, int64_t* capacity) {
    g_err.clear();
    if (!map_ok(map)) return state_err("invalid voxel map");
    if (level < 0 || level >= map->L) return invalid("level out of range");
    if (n_voxels) *n_voxels = map->lv[level].V;
    if (capacity) *capacity = (int64_t)1 << map->lv[level].log2cap;
    return VG_OK;
}

extern "C" vg_status vg_voxelmap_export(const vg_voxelmap* map, int32_t level, int64_t* n_voxels, int64_t* keys,
                                        double* means, double* covs, int64_t* counts) {
    g_err.clear();
    if (!map_ok(map)) return state_err("invalid voxel map");
    if (level < 0 || level >= map->L) return invalid("level out of range");
    if (n_voxels == nullptr) return invalid("n_voxels is NULL");
    const int64_t V = map->lv[level].V;
    if (*n_voxels < V) {
        *n_voxels = V;
        return invalid("output capacity too small");
    }
    *n_voxels = V;
    VG_HIP(hipSetDevice(map->ctx->device));
    return export_level(map->ctx, map->lv[level], keys, means, covs, counts);
}

extern "C" vg_status vg_voxelmap_destroy(vg_voxelmap* map) {
    g_err.clear();
    if (!map_ok(map)) return state_err("invalid voxel map");
    if (map->users > 0) return state_err("voxel map is used by a live batch");
    (void)hipSetDevice(map->ctx->device);
    (void)hipStreamSynchronize(map->ctx->stream);
    for (int l = 0; l < kMaxLevels; ++l) free_level(&map->lv[l]);
    map->magic = 0;
    delete map;
    return VG_OK;
}

// ============================================================================ sources

static void free_source(vg_source* s) {
    dfree(s->dxyz);
    dfree(s->cov);
    dfree(s->nrm);
    dfree(s->anchor);
    dfree(s->cbound);
    dfree(s->axyz);
    dfree(s->xyz64);
    dfree(s->cov64);
    dfree(s->nrm64);
    dfree(s->perm);
}

// Upper bound of |mu - origin| over a source's points from its chunk anchors
// and ball radii (host copy of both; synchronizes the context stream).
static vg_status source_extent(vg_context* ctx, vg_source* s) {
    std::vector<double> an(3 * s->n_chunks);
    std::vector<float> cb(8 * s->n_chunks);
    VG_HIP(hipMemcpyAsync(an.data(), s->anchor, sizeof(double) * an.size(), hipMemcpyDeviceToHost, ctx->stream));
    VG_HIP(hipMemcpyAsync(cb.data(), s->cbound, sizeof(float) * cb.size(), hipMemcpyDeviceToHost, ctx->stream));
    VG_HIP(hipStreamSynchronize(ctx->stream));
    double ext = 0.0;
    for (int64_t c = 0; c < s->n_chunks; ++c) {
        const double dx = an[3 * c] - s->origin[0], dy = an[3 * c + 1] - s->origin[1], dz = an[3 * c + 2] - s->origin[2];
        ext = std::max(ext, std::sqrt(dx * dx + dy * dy + dz * dz) + (double)cb[8 * c + 3]);
    }
    s->extent = ext;
    return VG_OK;
}

// Source from device FP64 arrays (caller order); first = host copy of point 0.
static vg_status make_source(vg_context* ctx, const double* d_xyz, const double* d_cov, const double* d_nrm,
                             bool has_normals, int64_t n, const double* first, vg_source** out) {
    auto* s = new vg_source();
    s->ctx = ctx;
    s->n = n;
    s->n_pad = ((n + kChunk - 1) / kChunk) * kChunk;
    s->n_chunks = s->n_pad / kChunk;
    s->has_normals = has_normals;
    for (int a = 0; a < 3; ++a) s->origin[a] = (n > 0) ? std::nearbyint(first[a]) : 0.0;
    const int64_t np = s->n_pad;
    vg_status st = VG_OK;
    do {
        if ((st = dev_alloc(&s->dxyz, 3 * np)) != VG_OK) break;
        if ((st = dev_alloc(&s->cov, 6 * np)) != VG_OK) break;
        if ((st = dev_alloc(&s->anchor, 3 * s->n_chunks)) != VG_OK) break;
        if ((st = dev_alloc(&s->cbound, 8 * s->n_chunks)) != VG_OK) break;
        if ((st = dev_alloc(&s->axyz, 3 * np)) != VG_OK) break;
        if ((st = dev_alloc(&s->xyz64, 3 * np)) != VG_OK) break;
        if ((st = dev_alloc(&s->cov64, 6 * np)) != VG_OK) break;
        if ((st = dev_alloc(&s->perm, np)) != VG_OK) break;
        if (has_normals) {
            if ((st = dev_alloc(&s->nrm, 3 * np)) != VG_OK) break;
            if ((st = dev_alloc(&s->nrm64, 3 * np)) != VG_OK) break;
        }
        if (n == 0) break;
        if ((st = layout_source(ctx, s, d_xyz, d_cov, d_nrm)) != VG_OK) break;
        st = source_extent(ctx, s);
    } while (0);
    if (st != VG_OK) {
        free_source(s);
        delete s;
        return st;
    }
    s->magic = kSrcMagic;
    *out = s;
    return VG_OK;
}

extern "C" vg_status vg_create_source(vg_context* ctx, const double* xyz, const double* cov, const double* normals,
                                      int64_t n, vg_source** out) {
    g_err.clear();
    const TimelineRange range_("vg_create_source");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    if (n < 0) return invalid("n < 0");
    if (n >= (int64_t)1 << 27) return invalid("n must be below 2^27 (134,217,728 points per source)");
    if (n > 0 && (xyz == nullptr || cov == nullptr)) return invalid("xyz or cov is NULL");
    if (n > 0 && !finite_all(xyz, 3 * n)) return invalid("xyz has non-finite values");
    if (n > 0 && !finite_all(cov, 6 * n)) return invalid("cov has non-finite values");
    if (n > 0 && normals && !finite_all(normals, 3 * n)) return invalid("normals have non-finite values");
    for (int64_t i = 0; i < n; ++i)
        if (!spd6(cov + 6 * i)) {
            set_error("covariance of point " + std::to_string(i) + " is not SPD");
            return VG_ERR_NOT_SPD;
        }
    VG_HIP(hipSetDevice(ctx->device));
    double *d_xyz = nullptr, *d_cov = nullptr, *d_nrm = nullptr;
    vg_status st = VG_OK;
    do {
        if (n == 0) {
            st = make_source(ctx, nullptr, nullptr, nullptr, normals != nullptr, 0, xyz, out);
            break;
        }
        if ((st = dev_alloc(&d_xyz, 3 * n)) != VG_OK) break;
        if ((st = dev_alloc(&d_cov, 6 * n)) != VG_OK) break;
        if (normals && (st = dev_alloc(&d_nrm, 3 * n)) != VG_OK) break;
        hipError_t e = hipMemcpyAsync(d_xyz, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(d_cov, cov, sizeof(double) * 6 * n, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess && normals)
            e = hipMemcpyAsync(d_nrm, normals, sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) {
            st = hip_fail(e, "source upload");
            break;
        }
        st = make_source(ctx, d_xyz, d_cov, d_nrm, normals != nullptr, n, xyz, out);
    } while (0);
    dfree(d_xyz);
    dfree(d_cov);
    dfree(d_nrm);
    return st;
}

extern "C" vg_status vg_source_set_points_async(vg_source* src, const void* d_xyz, int32_t dtype) {
    g_err.clear();
    const TimelineRange range_("vg_source_set_points_async");
    if (!src_ok(src)) return state_err("invalid source");
    if (dtype != 0 && dtype != 1) return invalid("dtype must be 0 (float32) or 1 (float64)");
    if (src->n > 0 && d_xyz == nullptr) return invalid("d_xyz is NULL");
    VG_HIP(hipSetDevice(src->ctx->device));
    return set_source_points(src->ctx, src, d_xyz, dtype);
}

extern "C" vg_status vg_source_destroy(vg_source* src) {
    g_err.clear();
    if (!src_ok(src)) return state_err("invalid source");
    if (src->users > 0) return state_err("source is used by a live batch");
    (void)hipSetDevice(src->ctx->device);
    (void)hipStreamSynchronize(src->ctx->stream);
    free_source(src);
    src->magic = 0;
    delete src;
    return VG_OK;
}

// ============================================================================ preprocessed clouds

static constexpr uint32_t kCloudMagic = 0xC10D0001u;
static bool cloud_ok(const vg_cloud* c) { return c != nullptr && c->magic == kCloudMagic; }

extern "C" vg_status vg_preprocess(vg_context* ctx, const double* xyz, int64_t n, double r, int32_t k,
                                   const double* sensor, vg_cloud** out) {
    g_err.clear();
    const TimelineRange range_("vg_preprocess");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    if (n < 0) return invalid("n < 0");
    if (n >= (int64_t)1 << 31) return invalid("n must be below 2^31");
    if (n > 0 && xyz == nullptr) return invalid("xyz is NULL");
    if (!(std::isfinite(r) && r > 0.0)) return invalid("r must be positive and finite");
    if (k < 1 || k > 32) return invalid("k must be in 1..32");
    if (sensor == nullptr || !finite_all(sensor, 3)) return invalid("sensor must be 3 finite values");
    if (n > 0 && !finite_all(xyz, 3 * n)) return invalid("xyz has non-finite values");
    VG_HIP(hipSetDevice(ctx->device));
    double* d_xyz = nullptr;
    auto* c = new vg_cloud();
    c->ctx = ctx;
    vg_status st = VG_OK;
    do {
        if ((st = dev_alloc(&d_xyz, 3 * n)) != VG_OK) break;
        if (n > 0) {
            hipError_t e = hipMemcpyAsync(d_xyz, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream);
            if (e != hipSuccess) {
                st = hip_fail(e, "frame upload");
                break;
            }
        }
        st = preprocess_frame(ctx, d_xyz, n, r, k, sensor, c);
    } while (0);
    dfree(d_xyz);
    if (st != VG_OK) {
        free_cloud(c);
        delete c;
        return st;
    }
    c->magic = kCloudMagic;
    *out = c;
    return VG_OK;
}

extern "C" vg_status vg_cloud_info(const vg_cloud* cloud, int64_t* n_points, int32_t* k) {
    g_err.clear();
    if (!cloud_ok(cloud)) return state_err("invalid cloud");
    if (n_points) *n_points = cloud->m;
    if (k) *k = cloud->k;
    return VG_OK;
}

extern "C" vg_status vg_cloud_export(const vg_cloud* cloud, double* xyz, double* cov, double* cov_raw,
                                     double* normals, int64_t* counts, int32_t* nbr, double* nbr_d2) {
    g_err.clear();
    if (!cloud_ok(cloud)) return state_err("invalid cloud");
    VG_HIP(hipSetDevice(cloud->ctx->device));
    hipStream_t st = cloud->ctx->stream;
    const int64_t m = cloud->m, k = cloud->k;
    if (m == 0) return VG_OK;
    if (xyz) VG_HIP(hipMemcpyAsync(xyz, cloud->xyz, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, st));
    if (cov) VG_HIP(hipMemcpyAsync(cov, cloud->cov, sizeof(double) * 6 * m, hipMemcpyDeviceToHost, st));
    if (cov_raw) VG_HIP(hipMemcpyAsync(cov_raw, cloud->cov_raw, sizeof(double) * 6 * m, hipMemcpyDeviceToHost, st));
    if (normals) VG_HIP(hipMemcpyAsync(normals, cloud->nrm, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, st));
    if (nbr) VG_HIP(hipMemcpyAsync(nbr, cloud->nbr, sizeof(int32_t) * m * k, hipMemcpyDeviceToHost, st));
    if (nbr_d2) VG_HIP(hipMemcpyAsync(nbr_d2, cloud->d2, sizeof(double) * m * k, hipMemcpyDeviceToHost, st));
    std::vector<int32_t> c32;
    if (counts) {
        c32.resize(m);
        VG_HIP(hipMemcpyAsync(c32.data(), cloud->counts, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st));
    }
    VG_HIP(hipStreamSynchronize(st));
    if (counts)
        for (int64_t i = 0; i < m; ++i) counts[i] = c32[i];
    return VG_OK;
}

extern "C" vg_status vg_create_source_from_cloud(vg_context* ctx, const vg_cloud* cloud, vg_source** out) {
    g_err.clear();
    const TimelineRange range_("vg_create_source_from_cloud");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (!cloud_ok(cloud)) return state_err("invalid cloud");
    if (cloud->ctx != ctx) return state_err("cloud from another context");
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    VG_HIP(hipSetDevice(ctx->device));
    if (cloud->m >= (int64_t)1 << 27) return invalid("a source holds fewer than 2^27 points");
    return make_source(ctx, cloud->xyz, cloud->cov, cloud->nrm, true, cloud->m, cloud->first, out);
}

extern "C" vg_status vg_build_voxelmap_from_cloud(vg_context* ctx, const vg_cloud* cloud, const double* resolutions,
                                                  int32_t L, vg_voxelmap** out) {
    g_err.clear();
    const TimelineRange range_("vg_build_voxelmap_from_cloud");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (!cloud_ok(cloud)) return state_err("invalid cloud");
    if (cloud->ctx != ctx) return state_err("cloud from another context");
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    VG_TRY(check_resolutions(resolutions, L));
    VG_HIP(hipSetDevice(ctx->device));
    return make_voxelmap(ctx, cloud->xyz, cloud->cov, cloud->m, resolutions, L, cloud->first, out);
}

extern "C" vg_status vg_cloud_destroy(vg_cloud* cloud) {
    g_err.clear();
    if (!cloud_ok(cloud)) return state_err("invalid cloud");
    (void)hipSetDevice(cloud->ctx->device);
    (void)hipStreamSynchronize(cloud->ctx->stream);
    free_cloud(cloud);
    cloud->magic = 0;
    delete cloud;
    return VG_OK;
}

// ============================================================================ batches

namespace {

void fill_factor(vg_batch* b, int64_t f, const double* viewpoints) {
    const vg_source* s = b->src[f];
    const vg_voxelmap* m = b->tgt[f];
    FactorDesc d{};
    d.dxyz = s->dxyz;
    d.cov = s->cov;
    d.nrm = s->nrm;
    d.anchor = s->anchor;
    d.cbound = s->cbound;
    d.axyz = s->axyz;
    d.xyz64 = s->xyz64;
    d.cov64 = s->cov64;
    d.nrm64 = s->nrm64;
    d.perm = s->perm;
    d.n = s->n;
    d.n_pad = s->n_pad;
    d.L = m->L;
    for (int a = 0; a < 3; ++a) {
        d.src_origin[a] = s->origin[a];
        d.viewpoint[a] = viewpoints ? viewpoints[3 * f + a] : 0.0;
    }
    const double rmax = m->lv[m->L - 1].r;
    for (int l = 0; l < m->L; ++l) {
        const Level& lv = m->lv[l];
        LevelDesc& q = d.lv[l];
        q.slots = lv.slots;
        q.rec32 = lv.rec32;
        q.recN = lv.recN;
        q.rec64 = lv.rec64;
        q.log2cap = lv.log2cap;
        q.scale = (int32_t)std::llround(rmax / lv.r);
        q.log2scale = 0;
        while ((1 << q.log2scale) < q.scale) ++q.log2scale;
        q.r = (float)lv.r;
        q.inv_r = (float)(1.0 / lv.r);
        q.r64 = lv.r;
        q.inv_r64 = 1.0 / lv.r;
        for (int a = 0; a < 3; ++a) {
            q.K0[a] = lv.K0[a];
            q.kmin[a] = lv.kmin[a];
            q.kmax[a] = lv.kmax[a];
            const bool empty = lv.kmin[a] > lv.kmax[a];
            q.kbox0[a] = empty ? 0 : lv.kmin[a];
            q.kboxw[a] = empty ? 0u : (uint32_t)(lv.kmax[a] - lv.kmin[a]);
            q.blo[a] = empty ? 1e30 : (double)(lv.K0[a] + lv.kmin[a]) * lv.r;
            q.bhi[a] = empty ? -1e30 : (double)(lv.K0[a] + lv.kmax[a] + 1) * lv.r;
        }
    }
    b->h_fac[f] = d;
}

void build_tiles(vg_batch* b) {
    const int tc = std::max(1, b->tile_points / kChunk);
    b->h_tiles.clear();
    b->h_tile_first.assign(b->F + 1, 0);
    for (int64_t f = 0; f < b->F; ++f) {
        b->h_tile_first[f] = (int32_t)b->h_tiles.size();
        const int64_t nch = b->src[f]->n_chunks;
        for (int64_t c = 0; c < nch; c += tc) {
            Tile t{};
            t.factor = (int32_t)f;
            t.chunk0 = (int32_t)c;
            t.nchunks = (int32_t)std::min<int64_t>(tc, nch - c);
            b->h_tiles.push_back(t);
        }
    }
    b->h_tile_first[b->F] = (int32_t)b->h_tiles.size();
}

void free_graph(vg_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

vg_status upload_schedule(vg_batch* b) {
    hipStream_t st = b->ctx->stream;
    dfree(b->d_tiles);
    dfree(b->d_tile_first);
    dfree(b->d_partials);
    b->d_tiles = nullptr;
    b->d_tile_first = nullptr;
    b->d_partials = nullptr;
    const size_t nt = b->h_tiles.size();
    VG_TRY(dev_alloc(&b->d_tiles, nt));
    VG_TRY(dev_alloc(&b->d_tile_first, b->F + 1));
    VG_TRY(dev_alloc(&b->d_partials, (size_t)kRow * std::max<size_t>(nt, 1)));
    if (nt) VG_HIP(hipMemcpyAsync(b->d_tiles, b->h_tiles.data(), sizeof(Tile) * nt, hipMemcpyHostToDevice, st));
    VG_HIP(hipMemcpyAsync(b->d_tile_first, b->h_tile_first.data(), sizeof(int32_t) * (b->F + 1),
                          hipMemcpyHostToDevice, st));
    const int64_t want = (int64_t)b->ctx->num_cu * b->blocks_per_cu;
    b->grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)nt));
    VG_HIP(hipStreamSynchronize(st));
    free_graph(b);
    return VG_OK;
}

int default_blocks_per_cu(int block) { return std::max(1, 2048 / block); }

std::string tune_key(const vg_batch* b) {
    std::ostringstream k;
    // the device by architecture and compute-unit count (its marketing name is not
    // always available to the runtime)
    k << b->ctx->arch << "|cu" << b->ctx->num_cu << "|p" << b->opt.precision << "|F" << b->F << "|N"
      << b->total_points << "|L" << b->L << "|v" << b->opt.surface_validation;
    return k.str();
}

bool tune_lookup(const vg_batch* b, int* block, int* tile, int* bpc, int* order) {
    if (b->opt.tune_cache == nullptr) return false;
    std::ifstream in(b->opt.tune_cache);
    if (!in) return false;
    const std::string key = "\"key\": \"" + tune_key(b) + "\"";
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        if (line.find(key) == std::string::npos) continue;
        int bl = 0, tp = 0, bc = 0, to = 0;
        const char* p1 = std::strstr(line.c_str(), "\"block\": ");
        const char* p2 = std::strstr(line.c_str(), "\"tile_points\": ");
        const char* p3 = std::strstr(line.c_str(), "\"blocks_per_cu\": ");
        const char* p4 = std::strstr(line.c_str(), "\"tile_order\": ");
        if (p1 && p2 && p3 && p4 && std::sscanf(p1 + 9, "%d", &bl) == 1 && std::sscanf(p2 + 15, "%d", &tp) == 1 &&
            std::sscanf(p3 + 17, "%d", &bc) == 1 && std::sscanf(p4 + 14, "%d", &to) == 1) {
            *block = bl;
            *tile = tp;
            *bpc = bc;
            *order = to;
            found = true;   // last entry wins
        }
    }
    return found;
}

bool valid_shape(int block, int tile, int bpc) {
    return (block == 64 || block == 128 || block == 256 || block == 512) && tile >= kChunk && tile % kChunk == 0 &&
           tile <= kMaxTilePoints && bpc >= 1 && bpc <= 64;
}

// The batch's own buffers for the tile kernel and reduction.
Workspace batch_ws(vg_batch* b) { return Workspace{b->d_partials, b->d_counter, b->d_posef, b->d_work}; }

vg_status run_linearize_device(vg_batch* b, const Workspace& ws, const double* d_poses, double* d_out,
                               int64_t* d_inl) {
    const int32_t nt = (int32_t)b->h_tiles.size();
    VG_TRY(launch_tiles(b, ws, kLin, d_poses, 0, nt, b->grid, nullptr, nullptr, 0, 0, b->F));
    return launch_reduce(b, ws, kLin, d_poses, 0, (int32_t)b->F, d_out, d_inl, nullptr, nullptr, nullptr);
}

vg_status run_linearize_device(vg_batch* b, const double* d_poses, double* d_out, int64_t* d_inl) {
    return run_linearize_device(b, batch_ws(b), d_poses, d_out, d_inl);
}

vg_status run_evaluate_device(vg_batch* b, const double* d_poses, double* d_e) {
    const int32_t nt = (int32_t)b->h_tiles.size();
    const Workspace ws = batch_ws(b);
    VG_TRY(launch_tiles(b, ws, kEval, d_poses, 0, nt, b->grid, nullptr, nullptr, 0, 0, b->F));
    return launch_reduce(b, ws, kEval, d_poses, 0, (int32_t)b->F, d_e, nullptr, nullptr, nullptr, nullptr);
}

// Capture [H2D poses, tile kernel, reduction, D2H results] once; replayed per call.
vg_status ensure_graph(vg_batch* b) {
    if (b->exec) return VG_OK;
    hipStream_t cs = nullptr;
    VG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t saved = b->ctx->stream;
    b->ctx->stream = cs;
    vg_status st = VG_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * b->F, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) st = run_linearize_device(b, b->d_poses, b->d_out, b->d_inliers);
        if (e == hipSuccess && st == VG_OK)
            e = hipMemcpyAsync(b->h_out, b->d_out, sizeof(double) * kOutRow * b->F, hipMemcpyDeviceToHost, cs);
        if (e == hipSuccess && st == VG_OK)
            e = hipMemcpyAsync(b->h_inliers, b->d_inliers, sizeof(int64_t) * b->L * b->F, hipMemcpyDeviceToHost, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        b->graph = g;
        if (e == hipSuccess && st == VG_OK) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    }
    b->ctx->stream = saved;
    (void)hipStreamDestroy(cs);
    if (st != VG_OK) {
        free_graph(b);
        return st;
    }
    if (e != hipSuccess) {
        free_graph(b);
        return hip_fail(e, "graph capture");
    }
    return VG_OK;
}

// The whole host-side linearize: stage poses, run, fetch results (pinned buffers).
vg_status linearize_host(vg_batch* b) {
    hipStream_t st = b->ctx->stream;
    const int64_t F = b->F;
    if (b->opt.plain_per_factor) {
        for (int64_t f = 0; f < F; ++f) {
            VG_HIP(hipMemcpyAsync(b->d_poses + 12 * f, b->h_poses + 12 * f, sizeof(double) * 12,
                                  hipMemcpyHostToDevice, st));
            const int32_t t0 = b->h_tile_first[f], t1 = b->h_tile_first[f + 1];
            const int grid = std::max(1, std::min(t1 - t0, b->grid));
            const Workspace ws = batch_ws(b);
            VG_TRY(launch_tiles(b, ws, kLin, b->d_poses, t0, t1, grid, nullptr, nullptr, 0, f, f + 1));
            VG_TRY(launch_reduce(b, ws, kLin, b->d_poses, (int32_t)f, (int32_t)f + 1, b->d_out, b->d_inliers,
                                 nullptr, nullptr, nullptr));
            VG_HIP(hipMemcpyAsync(b->h_out + kOutRow * f, b->d_out + kOutRow * f, sizeof(double) * kOutRow,
                                  hipMemcpyDeviceToHost, st));
            VG_HIP(hipMemcpyAsync(b->h_inliers + b->L * f, b->d_inliers + b->L * f, sizeof(int64_t) * b->L,
                                  hipMemcpyDeviceToHost, st));
            VG_HIP(hipStreamSynchronize(st));
        }
        return VG_OK;
    }
    if (b->opt.use_graph) {
        VG_TRY(ensure_graph(b));
        VG_HIP(hipGraphLaunch(b->exec, st));
        VG_HIP(hipStreamSynchronize(st));
        return VG_OK;
    }
    VG_HIP(hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * F, hipMemcpyHostToDevice, st));
    VG_TRY(run_linearize_device(b, b->d_poses, b->d_out, b->d_inliers));
    VG_HIP(hipMemcpyAsync(b->h_out, b->d_out, sizeof(double) * kOutRow * F, hipMemcpyDeviceToHost, st));
    VG_HIP(hipMemcpyAsync(b->h_inliers, b->d_inliers, sizeof(int64_t) * b->L * F, hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    return VG_OK;
}

void free_batch(vg_batch* b) {
    free_graph(b);
    dfree(b->d_fac);
    dfree(b->d_tiles);
    dfree(b->d_tile_first);
    dfree(b->d_partials);
    dfree(b->d_counter);
    dfree(b->d_poses);
    dfree(b->d_posef);
    dfree(b->d_out);
    dfree(b->d_inliers);
    dfree(b->d_work);
    dfree(b->d_e);
    dfree(b->d_lm);
    dfree(b->d_shared);
    dfree(b->d_slab_off);
    dfree(b->d_gslab);
    hfree(b->h_poses);
    hfree(b->h_out);
    hfree(b->h_inliers);
}

}  // namespace

extern "C" vg_status vg_create_factor_batch(vg_context* ctx, int64_t F, vg_source* const* src,
                                            vg_voxelmap* const* tgt, const double* target_viewpoints,
                                            const vg_batch_options* opts, vg_batch** out) {
    g_err.clear();
    const TimelineRange range_("vg_create_factor_batch");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (out == nullptr) return invalid("out is NULL");
    *out = nullptr;
    if (F < 1) return invalid("F must be >= 1");
    if (F >= (int64_t)1 << 30) return invalid("F too large");
    if (src == nullptr || tgt == nullptr) return invalid("src or tgt is NULL");
    vg_batch_options o{};
    if (opts) o = *opts;
    if (o.precision < 0 || o.precision > 2) return invalid("unknown precision");
    if (target_viewpoints && !finite_all(target_viewpoints, 3 * F)) return invalid("viewpoints are not finite");
    int L = -1;
    for (int64_t f = 0; f < F; ++f) {
        if (!src_ok(src[f])) return state_err("factor " + std::to_string(f) + ": invalid source");
        if (!map_ok(tgt[f])) return state_err("factor " + std::to_string(f) + ": invalid voxel map");
        if (src[f]->ctx != ctx || tgt[f]->ctx != ctx) return state_err("handle from another context");
        if (L < 0) L = tgt[f]->L;
        if (tgt[f]->L != L) return invalid("all voxel maps of a batch need the same number of levels");
        if (o.surface_validation && !src[f]->has_normals)
            return invalid("surface validation needs sources created with normals");
        if (src[f]->n_chunks > ((int64_t)1 << 31) / 2) return invalid("source too large");
    }
    int block = o.block_threads ? o.block_threads : 256;
    int tile = o.tile_points ? o.tile_points : 2048;
    int bpc = o.blocks_per_cu ? o.blocks_per_cu : default_blocks_per_cu(block);
    if (!valid_shape(block, tile, bpc)) return invalid("invalid launch shape (block 64/128/256/512, tile a multiple of 64 up to 32768)");
    if (o.tile_order < 0 || o.tile_order > 2) return invalid("tile_order must be 0, 1 or 2");
    if (o.precision == kC32) {
        for (int64_t f = 0; f < F; ++f)
            if (src[f]->extent > kMaxCompensatedExtent) {
                char msg[320];
                std::snprintf(msg, sizeof msg,
                              "factor %lld: source spans %.1f m from its origin; the compensated FP32 mode keeps "
                              "lever arms in FP32 and is limited to %.0f m (relative error of b above 1e-5 "
                              "beyond); use VG_FP64 or split the cloud",
                              (long long)f, src[f]->extent, kMaxCompensatedExtent);
                return invalid(msg);
            }
    }
    VG_HIP(hipSetDevice(ctx->device));
    auto* b = new vg_batch();
    b->ctx = ctx;
    b->F = F;
    b->L = L;
    b->opt = o;
    b->opt.tune_cache = nullptr;
    b->src.assign(src, src + F);
    b->tgt.assign(tgt, tgt + F);
    b->h_fac.resize(F);
    // concatenated point-gradient rows: sources in order of first use
    std::map<const vg_source*, std::pair<int64_t, int>> seen;
    int64_t rows = 0;
    for (int64_t f = 0; f < F; ++f) {
        auto it = seen.find(src[f]);
        if (it == seen.end()) {
            seen[src[f]] = {rows, 1};
            rows += src[f]->n;
        } else {
            it->second.second += 1;
        }
        b->total_points += src[f]->n;
    }
    b->grad_rows = rows;
    // sources used by several factors: each such factor writes its own point-gradient
    // rows, summed per source in factor order (the sources in order of first use)
    std::map<const vg_source*, size_t> shared_idx;
    for (int64_t f = 0; f < F; ++f) {
        fill_factor(b, f, target_viewpoints);
        b->h_fac[f].grad_offset = seen[src[f]].first;
        b->h_fac[f].grad_slab = -1;
        if (seen[src[f]].second > 1 && shared_idx.find(src[f]) == shared_idx.end()) {
            shared_idx[src[f]] = b->h_shared.size();
            SharedSrc q{};
            q.row0 = b->shared_rows;
            q.n = src[f]->n;
            q.grad_offset = seen[src[f]].first;
            b->h_shared.push_back(q);
            b->shared_rows += src[f]->n;
        }
        b->max_source_extent = std::max(b->max_source_extent, src[f]->extent);
    }
    if (!b->h_shared.empty()) {
        std::vector<std::vector<int64_t>> per(b->h_shared.size());
        for (int64_t f = 0; f < F; ++f) {
            auto it = shared_idx.find(src[f]);
            if (it == shared_idx.end()) continue;
            b->h_fac[f].grad_slab = b->slab_rows;
            per[it->second].push_back(b->slab_rows);
            b->slab_rows += src[f]->n;
        }
        for (size_t k = 0; k < per.size(); ++k) {
            b->h_shared[k].f0 = (int32_t)b->h_slab_off.size();
            b->h_slab_off.insert(b->h_slab_off.end(), per[k].begin(), per[k].end());
            b->h_shared[k].f1 = (int32_t)b->h_slab_off.size();
        }
    }
    b->block = block;
    b->tile_points = tile;
    b->blocks_per_cu = bpc;
    b->tile_order = o.tile_order ? o.tile_order : 1;
    if (opts && opts->tune_cache) {
        b->opt.tune_cache = strdup(opts->tune_cache);
        int bl = 0, tp = 0, bc = 0, to = 0;
        if (!o.block_threads && !o.tile_points && !o.blocks_per_cu && !o.tile_order &&
            tune_lookup(b, &bl, &tp, &bc, &to) && valid_shape(bl, tp, bc) && (to == 1 || to == 2)) {
            b->block = bl;
            b->tile_points = tp;
            b->blocks_per_cu = bc;
            b->tile_order = to;
        }
    }
    build_tiles(b);
    vg_status st = VG_OK;
    do {
        if ((st = dev_alloc(&b->d_fac, F)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_counter, 64)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_poses, 12 * F)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_posef, 16 * F)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_out, kOutRow * F)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_inliers, (size_t)L * F)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_work, (size_t)kWork * F)) != VG_OK) break;
        if (!b->h_shared.empty()) {
            if ((st = dev_alloc(&b->d_shared, b->h_shared.size())) != VG_OK) break;
            if ((st = dev_alloc(&b->d_slab_off, b->h_slab_off.size())) != VG_OK) break;
            hipError_t e1 = hipMemcpyAsync(b->d_shared, b->h_shared.data(), sizeof(SharedSrc) * b->h_shared.size(),
                                           hipMemcpyHostToDevice, ctx->stream);
            if (e1 == hipSuccess)
                e1 = hipMemcpyAsync(b->d_slab_off, b->h_slab_off.data(), sizeof(int64_t) * b->h_slab_off.size(),
                                    hipMemcpyHostToDevice, ctx->stream);
            if (e1 != hipSuccess) {
                st = hip_fail(e1, "shared-source table upload");
                break;
            }
        }
        if ((st = dev_alloc(&b->d_e, F)) != VG_OK) break;
        if ((st = dev_alloc(&b->d_lm, 32 * F)) != VG_OK) break;
        if ((st = host_alloc(&b->h_poses, 12 * F)) != VG_OK) break;
        if ((st = host_alloc(&b->h_out, kOutRow * F)) != VG_OK) break;
        if ((st = host_alloc(&b->h_inliers, (size_t)L * F)) != VG_OK) break;
        hipError_t e = hipMemcpyAsync(b->d_fac, b->h_fac.data(), sizeof(FactorDesc) * F, hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e != hipSuccess) {
            st = hip_fail(e, "factor table upload");
            break;
        }
        if ((st = launch_zero(ctx, b->d_counter, 64 * sizeof(uint32_t))) != VG_OK) break;
        if ((st = launch_zero(ctx, b->d_work, sizeof(int64_t) * kWork * F)) != VG_OK) break;
        st = upload_schedule(b);
    } while (0);
    if (st != VG_OK) {
        free_batch(b);
        if (b->opt.tune_cache) free((void*)b->opt.tune_cache);
        delete b;
        return st;
    }
    for (int64_t f = 0; f < F; ++f) {
        src[f]->users += 1;
        tgt[f]->users += 1;
    }
    b->magic = kBatMagic;
    *out = b;
    return VG_OK;
}

extern "C" vg_status vg_batch_info(const vg_batch* b, int64_t* total_points, int64_t* n_tiles, int32_t* block_threads,
                                   int32_t* tile_points, int32_t* grid_blocks, int32_t* tile_order) {
    g_err.clear();
    if (!bat_ok(b)) return state_err("invalid batch");
    if (total_points) *total_points = b->total_points;
    if (n_tiles) *n_tiles = (int64_t)b->h_tiles.size();
    if (block_threads) *block_threads = b->block;
    if (tile_points) *tile_points = b->tile_points;
    if (grid_blocks) *grid_blocks = b->grid;
    if (tile_order) *tile_order = b->tile_order;
    return VG_OK;
}

extern "C" vg_status vg_batch_destroy(vg_batch* b) {
    g_err.clear();
    if (!bat_ok(b)) return state_err("invalid batch");
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    for (int64_t f = 0; f < b->F; ++f) {
        b->src[f]->users -= 1;
        b->tgt[f]->users -= 1;
    }
    free_batch(b);
    if (b->opt.tune_cache) free((void*)b->opt.tune_cache);
    b->magic = 0;
    delete b;
    return VG_OK;
}

extern "C" vg_status vg_linearize(vg_batch* b, const double* poses, double* e, double* H, double* bv,
                                  int64_t* inliers) {
    g_err.clear();
    const TimelineRange range_("vg_linearize");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (e == nullptr || H == nullptr || bv == nullptr) return invalid("e, H or b is NULL");
    VG_TRY(check_poses(poses, b->F));
    VG_HIP(hipSetDevice(b->ctx->device));
    std::memcpy(b->h_poses, poses, sizeof(double) * 12 * b->F);
    VG_TRY(linearize_host(b));
    for (int64_t f = 0; f < b->F; ++f) {
        const double* r = b->h_out + kOutRow * f;
        e[f] = r[0];
        std::memcpy(H + 36 * f, r + 1, sizeof(double) * 36);
        std::memcpy(bv + 6 * f, r + 37, sizeof(double) * 6);
    }
    if (inliers) std::memcpy(inliers, b->h_inliers, sizeof(int64_t) * b->L * b->F);
    return VG_OK;
}

extern "C" vg_status vg_evaluate(vg_batch* b, const double* poses, double* e) {
    g_err.clear();
    const TimelineRange range_("vg_evaluate");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (e == nullptr) return invalid("e is NULL");
    VG_TRY(check_poses(poses, b->F));
    VG_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    std::memcpy(b->h_poses, poses, sizeof(double) * 12 * b->F);
    VG_HIP(hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * b->F, hipMemcpyHostToDevice, st));
    VG_TRY(run_evaluate_device(b, b->d_poses, b->d_e));
    VG_HIP(hipMemcpyAsync(b->h_out, b->d_e, sizeof(double) * b->F, hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    std::memcpy(e, b->h_out, sizeof(double) * b->F);
    return VG_OK;
}

extern "C" vg_status vg_overlap(vg_batch* b, const double* poses, double* overlap) {
    g_err.clear();
    const TimelineRange range_("vg_overlap");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (overlap == nullptr) return invalid("overlap is NULL");
    VG_TRY(check_poses(poses, b->F));
    VG_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    std::memcpy(b->h_poses, poses, sizeof(double) * 12 * b->F);
    VG_HIP(hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * b->F, hipMemcpyHostToDevice, st));
    const int32_t nt = (int32_t)b->h_tiles.size();
    const Workspace ws = batch_ws(b);
    VG_TRY(launch_tiles(b, ws, kCount, b->d_poses, 0, nt, b->grid, nullptr, nullptr, 0, 0, b->F));
    // the per-level fractions land in d_out (F x L <= F x 43)
    VG_TRY(launch_reduce(b, ws, kCount, b->d_poses, 0, (int32_t)b->F, b->d_out, nullptr, nullptr, nullptr, nullptr));
    VG_HIP(hipMemcpyAsync(b->h_out, b->d_out, sizeof(double) * b->L * b->F, hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    std::memcpy(overlap, b->h_out, sizeof(double) * b->L * b->F);
    return VG_OK;
}

extern "C" vg_status vg_linearize_async(vg_batch* b, const double* d_poses, double* d_out, int64_t* d_inliers) {
    g_err.clear();
    const TimelineRange range_("vg_linearize_async");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (d_poses == nullptr || d_out == nullptr) return invalid("d_poses or d_out is NULL");
    VG_HIP(hipSetDevice(b->ctx->device));
    return run_linearize_device(b, d_poses, d_out, d_inliers);
}

extern "C" vg_status vg_linearize_noalloc(vg_batch* b, const double* d_poses, double* d_out, int64_t* d_inliers) {
    g_err.clear();
    const TimelineRange range_("vg_linearize_noalloc");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (d_poses == nullptr || d_out == nullptr) return invalid("d_poses or d_out is NULL");
    VG_HIP(hipSetDevice(b->ctx->device));
    if (b->ctx->scratch == nullptr) {
        const int dev = b->ctx->device;
        set_error(std::string("no fixed scratch on this device: ") +
                  (dev < kMaxDevices ? hipGetErrorString(g_scratch_err[dev]) : "device index beyond the table"));
        return VG_ERR_HIP;
    }
    // layout: counters (256 B), staged poses (F x 16 floats), tile rows (tiles x kRow doubles)
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t n_tiles = b->h_tiles.size();
    const size_t off_posef = 256;
    const size_t off_rows = off_posef + up(sizeof(float) * 16 * (size_t)b->F);
    const size_t need = off_rows + up(sizeof(double) * kRow * n_tiles);
    if (need > kScratchBytes) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "batch needs %zu bytes of scratch (%lld factors, %zu tiles); the fixed scratch holds %zu",
                      need, (long long)b->F, n_tiles, kScratchBytes);
        set_error(msg);
        return VG_ERR_CAPACITY;
    }
    unsigned char* base = static_cast<unsigned char*>(b->ctx->scratch);
    const Workspace ws{reinterpret_cast<double*>(base + off_rows), reinterpret_cast<uint32_t*>(base),
                       reinterpret_cast<float*>(base + off_posef), nullptr};
    // the tile counters must start at zero; another call may have left them anywhere
    VG_TRY(launch_zero(b->ctx, ws.counter, sizeof(uint32_t) * kParts));
    return run_linearize_device(b, ws, d_poses, d_out, d_inliers);
}

extern "C" vg_status vg_evaluate_async(vg_batch* b, const double* d_poses, double* d_e) {
    g_err.clear();
    const TimelineRange range_("vg_evaluate_async");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (d_poses == nullptr || d_e == nullptr) return invalid("d_poses or d_e is NULL");
    VG_HIP(hipSetDevice(b->ctx->device));
    return run_evaluate_device(b, d_poses, d_e);
}

extern "C" vg_status vg_backward_async(vg_batch* b, const double* d_poses, const double* d_grad_e, const double* d_jr,
                                       double* d_grad_xi, void* d_grad_points, int32_t points_dtype) {
    g_err.clear();
    const TimelineRange range_("vg_backward_async");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (d_poses == nullptr || d_grad_e == nullptr || d_grad_xi == nullptr)
        return invalid("d_poses, d_grad_e or d_grad_xi is NULL");
    if (points_dtype != 0 && points_dtype != 1) return invalid("points_dtype must be 0 or 1");
    VG_HIP(hipSetDevice(b->ctx->device));
    if (d_grad_points && b->slab_rows > 0) {
        // per-factor rows of the shared sources (allocated on first use, kept with the batch)
        const size_t need = (size_t)b->slab_rows * 3 * (points_dtype ? 8 : 4);
        if (b->gslab_bytes < need) {
            VG_HIP(hipStreamSynchronize(b->ctx->stream));
            dfree(b->d_gslab);
            b->d_gslab = nullptr;
            b->gslab_bytes = 0;
            unsigned char* p = nullptr;
            VG_TRY(dev_alloc(&p, need));
            b->d_gslab = p;
            b->gslab_bytes = need;
        }
    }
    if (d_grad_points) {
        VG_TRY(launch_zero(b->ctx, d_grad_points, (size_t)b->grad_rows * 3 * (points_dtype ? 8 : 4)));
        // the one-level compensated backward kernel writes only the rows of
        // points with a voxel, so the per-factor rows start at zero too
        const bool compacted = b->opt.precision == kC32 && !b->opt.lane_kahan && !b->opt.surface_validation &&
                               b->L == 1;
        if (compacted && b->slab_rows > 0)
            VG_TRY(launch_zero(b->ctx, b->d_gslab, (size_t)b->slab_rows * 3 * (points_dtype ? 8 : 4)));
    }
    const int32_t nt = (int32_t)b->h_tiles.size();
    const Workspace ws = batch_ws(b);
    VG_TRY(launch_tiles(b, ws, kBwd, d_poses, 0, nt, b->grid, d_grad_e, d_grad_points, points_dtype, 0, b->F));
    VG_TRY(launch_grad_combine(b, d_grad_points, points_dtype));
    return launch_reduce(b, ws, kBwd, d_poses, 0, (int32_t)b->F, nullptr, nullptr, d_grad_e, d_jr, d_grad_xi);
}

extern "C" vg_status vg_se3_retract_async(vg_context* ctx, int64_t F, const double* d_T0, const double* d_xi,
                                          double* d_T, double* d_jr) {
    g_err.clear();
    const TimelineRange range_("vg_se3_retract_async");
    if (!ctx_ok(ctx)) return state_err("invalid context");
    if (F < 0) return invalid("F < 0");
    if (F > 0 && (d_T0 == nullptr || d_xi == nullptr || d_T == nullptr)) return invalid("NULL pointer");
    VG_HIP(hipSetDevice(ctx->device));
    return launch_se3_retract(ctx, F, d_T0, d_xi, d_T, d_jr);
}

namespace {

// One Levenberg-Marquardt iteration for every factor, stream-ordered: linearize
// at d_poses, propose T Exp(delta) from (H + lambda diag H) delta = -b, evaluate
// the proposal, accept or reject it (lambda / 10 or x 10).  e at the input poses
// and the decision go to column `col` of d_e / d_acc (rows of `stride`).
vg_status lm_step(vg_batch* b, double* d_poses, double* d_lambda, double* d_e, int32_t* d_acc, int32_t stride,
                  int32_t col) {
    const int64_t F = b->F;
    double* cand = b->d_lm + F;                              // 12 per factor
    double* e_new = b->d_lm + 13 * F;                        // 1 per factor
    int32_t* valid = reinterpret_cast<int32_t*>(b->d_lm + 14 * F);
    VG_TRY(run_linearize_device(b, d_poses, b->d_out, nullptr));
    VG_TRY(launch_lm_propose(b, b->d_out, d_lambda, d_poses, cand, valid));
    VG_TRY(run_evaluate_device(b, cand, e_new));
    return launch_lm_accept(b, b->d_out, e_new, d_lambda, d_poses, cand, valid, d_e, d_acc, stride, col);
}

}  // namespace

extern "C" vg_status vg_lm_step_async(vg_batch* b, double* d_poses, double* d_lambda, double* d_e,
                                      int32_t* d_accepted) {
    g_err.clear();
    const TimelineRange range_("vg_lm_step_async");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (d_poses == nullptr || d_lambda == nullptr) return invalid("d_poses or d_lambda is NULL");
    VG_HIP(hipSetDevice(b->ctx->device));
    return lm_step(b, d_poses, d_lambda, d_e, d_accepted, 1, 0);
}

extern "C" vg_status vg_lm_run(vg_batch* b, const double* poses_in, int32_t iters, double lambda0, double* poses_out,
                               int32_t* accepted, double* e_hist) {
    g_err.clear();
    const TimelineRange range_("vg_lm_run");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (poses_out == nullptr) return invalid("poses_out is NULL");
    if (iters < 0 || iters > 10000) return invalid("iters out of range");
    if (!(std::isfinite(lambda0) && lambda0 > 0)) return invalid("lambda0 must be positive");
    VG_TRY(check_poses(poses_in, b->F));
    VG_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    const int64_t F = b->F;
    double* lambda = b->d_lm;                // 1 per factor
    int32_t* d_acc = nullptr;
    double* d_eh = nullptr;
    VG_TRY(dev_alloc(&d_acc, (size_t)F * std::max(iters, 1)));
    vg_status rc = dev_alloc(&d_eh, (size_t)F * std::max(iters, 1));
    if (rc != VG_OK) {
        dfree(d_acc);
        return rc;
    }
    do {
        std::memcpy(b->h_poses, poses_in, sizeof(double) * 12 * F);
        hipError_t e = hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * F, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            rc = hip_fail(e, "pose upload");
            break;
        }
        if ((rc = launch_fill(b->ctx, lambda, F, lambda0)) != VG_OK) break;
        for (int32_t it = 0; it < iters && rc == VG_OK; ++it) rc = lm_step(b, b->d_poses, lambda, d_eh, d_acc, iters, it);
        if (rc != VG_OK) break;
        std::vector<int32_t> ha((size_t)F * std::max(iters, 1));
        std::vector<double> he((size_t)F * std::max(iters, 1));
        e = hipMemcpyAsync(b->h_poses, b->d_poses, sizeof(double) * 12 * F, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && iters > 0)
            e = hipMemcpyAsync(ha.data(), d_acc, sizeof(int32_t) * F * iters, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && iters > 0)
            e = hipMemcpyAsync(he.data(), d_eh, sizeof(double) * F * iters, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            rc = hip_fail(e, "LM download");
            break;
        }
        std::memcpy(poses_out, b->h_poses, sizeof(double) * 12 * F);
        if (accepted && iters > 0) std::memcpy(accepted, ha.data(), sizeof(int32_t) * F * iters);
        if (e_hist && iters > 0) std::memcpy(e_hist, he.data(), sizeof(double) * F * iters);
    } while (0);
    dfree(d_acc);
    dfree(d_eh);
    return rc;
}

extern "C" vg_status vg_batch_work(vg_batch* b, int64_t* walked_points, int64_t* walked_chunks, int64_t* lookups) {
    g_err.clear();
    if (!bat_ok(b)) return state_err("invalid batch");
    VG_HIP(hipSetDevice(b->ctx->device));
    std::vector<int64_t> w((size_t)kWork * b->F);
    VG_HIP(hipMemcpyAsync(w.data(), b->d_work, sizeof(int64_t) * w.size(), hipMemcpyDeviceToHost, b->ctx->stream));
    VG_HIP(hipStreamSynchronize(b->ctx->stream));
    for (int64_t f = 0; f < b->F; ++f) {
        const int64_t* r = w.data() + kWork * f;
        if (walked_points) walked_points[f] = r[0];
        if (walked_chunks) walked_chunks[f] = r[1];
        if (lookups)
            for (int l = 0; l < b->L; ++l) lookups[(int64_t)b->L * f + l] = r[2 + l];
    }
    return VG_OK;
}

extern "C" vg_status vg_correspondences(vg_batch* b, const double* pose, int64_t factor, int64_t* keys,
                                        int32_t* found) {
    g_err.clear();
    const TimelineRange range_("vg_correspondences");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (factor < 0 || factor >= b->F) return invalid("factor out of range");
    if (keys == nullptr || found == nullptr) return invalid("keys or found is NULL");
    VG_TRY(check_poses(pose, 1));
    VG_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    const int64_t n = b->src[factor]->n, L = b->L;
    if (n == 0) return VG_OK;
    double* d_pose = nullptr;
    int64_t* d_keys = nullptr;
    int32_t* d_found = nullptr;
    vg_status rc = VG_OK;
    do {
        if ((rc = dev_alloc(&d_pose, 12)) != VG_OK) break;
        if ((rc = dev_alloc(&d_keys, (size_t)n * L * 3)) != VG_OK) break;
        if ((rc = dev_alloc(&d_found, (size_t)n * L)) != VG_OK) break;
        hipError_t e = hipMemcpyAsync(d_pose, pose, sizeof(double) * 12, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            rc = hip_fail(e, "pose upload");
            break;
        }
        if ((rc = launch_correspondences(b, d_pose, factor, d_keys, d_found)) != VG_OK) break;
        e = hipMemcpyAsync(keys, d_keys, sizeof(int64_t) * n * L * 3, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(found, d_found, sizeof(int32_t) * n * L, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "correspondence download");
    } while (0);
    dfree(d_pose);
    dfree(d_keys);
    dfree(d_found);
    return rc;
}

namespace {

// Average device time of the tile kernel and the reduction over `reps` launches.
vg_status time_device(vg_batch* b, int reps, float* ms_tiles, float* ms_reduce) {
    hipStream_t st = b->ctx->stream;
    const int32_t nt = (int32_t)b->h_tiles.size();
    std::vector<hipEvent_t> ev(3 * reps);
    for (auto& x : ev) VG_HIP(hipEventCreate(&x));
    vg_status rc = run_linearize_device(b, b->d_poses, b->d_out, b->d_inliers);   // warm-up
    for (int r = 0; r < reps && rc == VG_OK; ++r) {
        (void)hipEventRecord(ev[3 * r], st);
        rc = launch_tiles(b, batch_ws(b), kLin, b->d_poses, 0, nt, b->grid, nullptr, nullptr, 0, 0, b->F);
        (void)hipEventRecord(ev[3 * r + 1], st);
        if (rc == VG_OK)
            rc = launch_reduce(b, batch_ws(b), kLin, b->d_poses, 0, (int32_t)b->F, b->d_out, b->d_inliers, nullptr,
                               nullptr, nullptr);
        (void)hipEventRecord(ev[3 * r + 2], st);
    }
    hipError_t e = hipStreamSynchronize(st);
    float t1 = 0.f, t2 = 0.f;
    if (rc == VG_OK && e == hipSuccess) {
        for (int r = 0; r < reps; ++r) {
            float a = 0.f, c = 0.f;
            (void)hipEventElapsedTime(&a, ev[3 * r], ev[3 * r + 1]);
            (void)hipEventElapsedTime(&c, ev[3 * r + 1], ev[3 * r + 2]);
            t1 += a;
            t2 += c;
        }
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rc != VG_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "timing synchronize");
    *ms_tiles = t1 / reps;
    *ms_reduce = t2 / reps;
    return VG_OK;
}

}  // namespace

extern "C" vg_status vg_batch_time_kernels(vg_batch* b, const double* poses, int32_t reps, float* ms) {
    g_err.clear();
    if (!bat_ok(b)) return state_err("invalid batch");
    if (ms == nullptr) return invalid("ms is NULL");
    if (reps < 1 || reps > 100000) return invalid("reps out of range");
    VG_TRY(check_poses(poses, b->F));
    VG_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    std::memcpy(b->h_poses, poses, sizeof(double) * 12 * b->F);
    VG_HIP(hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * b->F, hipMemcpyHostToDevice, st));
    VG_TRY(time_device(b, reps, &ms[0], &ms[1]));
    VG_TRY(linearize_host(b));   // warm-up (captures the graph if enabled)
    const auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps; ++r) VG_TRY(linearize_host(b));
    const auto t1 = std::chrono::steady_clock::now();
    ms[2] = (float)(std::chrono::duration<double, std::milli>(t1 - t0).count() / reps);
    return VG_OK;
}

extern "C" vg_status vg_batch_tune(vg_batch* b, const double* poses, int32_t reps, int32_t* chosen) {
    g_err.clear();
    const TimelineRange range_("vg_batch_tune");
    if (!bat_ok(b)) return state_err("invalid batch");
    if (reps < 1 || reps > 1000) return invalid("reps out of range");
    VG_TRY(check_poses(poses, b->F));
    VG_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    std::memcpy(b->h_poses, poses, sizeof(double) * 12 * b->F);
    VG_HIP(hipMemcpyAsync(b->d_poses, b->h_poses, sizeof(double) * 12 * b->F, hipMemcpyHostToDevice, st));
    {
        // a shape already recorded in the tune cache for this device and batch signature
        int bl = 0, tp = 0, bc = 0, to = 0;
        if (!b->opt.plain_per_factor && tune_lookup(b, &bl, &tp, &bc, &to) && valid_shape(bl, tp, bc) &&
            (to == 1 || to == 2)) {
            b->block = bl;
            b->tile_points = tp;
            b->blocks_per_cu = bc;
            b->tile_order = to;
            build_tiles(b);
            VG_TRY(upload_schedule(b));
            if (chosen) {
                chosen[0] = bl;
                chosen[1] = tp;
                chosen[2] = bc;
                chosen[3] = to;
            }
            return VG_OK;
        }
    }
    if (b->opt.plain_per_factor) {
        // the per-factor loop: every factor is its own launch, so its tiles must
        // be small enough to fill the device on their own; each candidate is
        // timed on the whole loop (uploads, launches, downloads, synchronizations)
        const int ptiles[] = {8192, 2048, 1024, 512, 256};
        const int pblocks[] = {256, 128};
        float best = 1e30f;
        int bb = b->block, bt = b->tile_points;
        for (int tp : ptiles)
            for (int bl : pblocks) {
                b->tile_points = tp;
                b->block = bl;
                b->blocks_per_cu = default_blocks_per_cu(bl);
                build_tiles(b);
                VG_TRY(upload_schedule(b));
                VG_TRY(linearize_host(b));   // warm-up
                const auto t0 = std::chrono::steady_clock::now();
                for (int r = 0; r < reps; ++r) VG_TRY(linearize_host(b));
                const float ms = (float)(std::chrono::duration<double, std::milli>(
                                             std::chrono::steady_clock::now() - t0).count() / reps);
                if (ms < best * 0.985f) {
                    best = ms;
                    bb = bl;
                    bt = tp;
                }
            }
        b->block = bb;
        b->tile_points = bt;
        b->blocks_per_cu = default_blocks_per_cu(bb);
        build_tiles(b);
        VG_TRY(upload_schedule(b));
        if (chosen) {
            chosen[0] = bb;
            chosen[1] = bt;
            chosen[2] = b->blocks_per_cu;
            chosen[3] = b->tile_order;
        }
        return VG_OK;
    }
    // candidates in order of preference: a later candidate replaces an earlier one
    // only when it is faster by more than 1.5 %, so timing noise does not flip the choice
    const int orders[] = {1, 2};
    // preference order: larger tiles first (fewer partial rows to reduce, fewer
    // counter atomics); a later shape replaces the incumbent only if 1.5 % faster
    const int tiles[] = {16384, 8192, 32768, 4096, 2048, 1024, 512, 256};
    const int blocks[] = {256, 128, 512};
    const int occ[] = {2, 1, 4};   // multiples of the full-occupancy workgroup count
    struct Cand {
        int tp, bl, bc, to;
        float ms;
    };
    std::vector<Cand> cands;   // in preference order
    auto apply = [&](const Cand& c) -> vg_status {
        if (b->tile_points != c.tp || b->h_tiles.empty()) {
            b->tile_points = c.tp;
            build_tiles(b);
            VG_TRY(upload_schedule(b));
        }
        b->tile_order = c.to;
        b->block = c.bl;
        b->blocks_per_cu = c.bc;
        b->grid = (int)std::max<int64_t>(
            1, std::min<int64_t>((int64_t)b->ctx->num_cu * b->blocks_per_cu, (int64_t)b->h_tiles.size()));
        return VG_OK;
    };
    for (int tp : tiles) {
        // the small tiles are for small batches (more tiles than workgroups);
        // a batch that fills the device with 1024-point tiles skips them
        if (tp < 1024 && b->total_points / tp > (int64_t)(1 << 20)) continue;
        for (int to : orders)
            for (int bl : blocks)
                for (int oc : occ) {
                    Cand c{tp, bl, std::max(1, oc * 1024 / bl), to, 0.f};
                    VG_TRY(apply(c));
                    float t1 = 0.f, t2 = 0.f;
                    VG_TRY(time_device(b, reps, &t1, &t2));
                    c.ms = t1 + t2;
                    cands.push_back(c);
                }
    }
    // the sweep's three fastest shapes are timed again, in three interleaved
    // rounds (so drifts of the clock hit all of them), and the choice is made
    // on those sums: the earliest in preference order unless a later one is
    // more than 1.5 % faster (a short sweep's noise exceeds that margin)
    std::vector<size_t> order(cands.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cands[x].ms < cands[y].ms; });
    std::vector<size_t> top(order.begin(), order.begin() + std::min<size_t>(3, order.size()));
    std::sort(top.begin(), top.end());   // back to preference order
    std::vector<float> sum(top.size(), 0.f);
    constexpr int kRounds = 3;
    for (int r = 0; r < kRounds; ++r)
        for (size_t k = 0; k < top.size(); ++k) {
            VG_TRY(apply(cands[top[k]]));
            float t1 = 0.f, t2 = 0.f;
            VG_TRY(time_device(b, reps, &t1, &t2));
            sum[k] += t1 + t2;
        }
    float best = 1e30f;
    int bb = b->block, bt = b->tile_points, bc = b->blocks_per_cu, bo = b->tile_order;
    for (size_t k = 0; k < top.size(); ++k) {
        const float ms = sum[k] / kRounds;
        if (ms < best * 0.985f) {
            best = ms;
            const Cand& c = cands[top[k]];
            bb = c.bl;
            bt = c.tp;
            bc = c.bc;
            bo = c.to;
        }
    }
    b->tile_order = bo;
    b->block = bb;
    b->tile_points = bt;
    b->blocks_per_cu = bc;
    build_tiles(b);
    VG_TRY(upload_schedule(b));
    if (chosen) {
        chosen[0] = bb;
        chosen[1] = bt;
        chosen[2] = bc;
        chosen[3] = bo;
    }
    if (b->opt.tune_cache) {
        std::ofstream outf(b->opt.tune_cache, std::ios::app);
        if (outf) {
            outf << "{\"key\": \"" << tune_key(b) << "\", \"block\": " << bb << ", \"tile_points\": " << bt
                 << ", \"blocks_per_cu\": " << bc << ", \"tile_order\": " << bo << ", \"ms\": " << best << "}\n";
        }
    }
    return VG_OK;
}
