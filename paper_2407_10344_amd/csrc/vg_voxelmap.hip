// Gaussian voxel map construction (GLIM Sec. III-C, Preprocessing): every point
// x falls in voxel floor(x / r); a voxel stores the average of its points' means
// and the average of their covariances.
//
// Device pipeline per level: FP64 keys -> stable radix sort of (key, point) ->
// run-length encoding -> one thread per voxel sums its run in ascending point
// order in FP64 (deterministic, identical summation order for every build) ->
// records in three layouts -> open-addressing insert with 64-bit atomicCAS.
#include <hipcub/hipcub.hpp>

#include <climits>

#include "vg_device.h"

namespace vg {

__global__ void k_level_keys(const double* __restrict__ xyz, int64_t n, double r, int64_t K0x, int64_t K0y,
                             int64_t K0z, uint64_t* __restrict__ keys, int32_t* __restrict__ idx,
                             int32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t kx = (int64_t)floor(xyz[3 * i + 0] / r) - K0x;
    const int64_t ky = (int64_t)floor(xyz[3 * i + 1] / r) - K0y;
    const int64_t kz = (int64_t)floor(xyz[3 * i + 2] / r) - K0z;
    if (!(key_in_range(kx) && key_in_range(ky) && key_in_range(kz))) {
        atomicOr(flag, 1);
        keys[i] = 0;
    } else {
        keys[i] = pack_key(kx, ky, kz);
    }
    idx[i] = (int32_t)i;
}

__global__ void k_level_stats(const double* __restrict__ xyz, const double* __restrict__ cov,
                              const uint64_t* __restrict__ ukeys, const int32_t* __restrict__ counts,
                              const int32_t* __restrict__ offsets, const int32_t* __restrict__ sorted_idx, int64_t V,
                              double r, int64_t K0x, int64_t K0y, int64_t K0z, float* __restrict__ rec32,
                              float* __restrict__ recN, double* __restrict__ rec64, uint64_t* __restrict__ keys_out,
                              int32_t* __restrict__ counts_out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int32_t off = offsets[v], cnt = counts[v];
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t j = off; j < off + cnt; ++j) {
        const int64_t i = sorted_idx[j];
        s[0] += xyz[3 * i + 0];
        s[1] += xyz[3 * i + 1];
        s[2] += xyz[3 * i + 2];
#pragma unroll
        for (int k = 0; k < 6; ++k) s[3 + k] += cov[6 * i + k];
    }
    double m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = s[k] / (double)cnt;
    const uint64_t key = ukeys[v];
    int64_t q[3];
    unpack_key(key, q);
    q[0] += K0x;
    q[1] += K0y;
    q[2] += K0z;
    double* r64 = rec64 + kRec64 * v;
    float* r32 = rec32 + kRec32 * v;
    float* rN = recN + kRecN * v;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double centre = (double)q[a] * r + 0.5 * r;
        r64[a] = m[a];
        r32[a] = (float)(m[a] - centre);
        rN[a] = (float)m[a];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float hi = (float)m[3 + k];
        r64[3 + k] = m[3 + k];
        r32[3 + k] = hi;                                // covariance, high part
        r32[9 + k] = (float)(m[3 + k] - (double)hi);    // covariance, low part
        rN[3 + k] = hi;
    }
    r64[9] = 0.0;
    r32[15] = (float)cnt;
    rN[9] = 0.f;
    rN[10] = 0.f;
    rN[11] = 0.f;
    keys_out[v] = key;
    counts_out[v] = cnt;
}

// Bounding box of the level's relative keys (box[0..2] = min, box[3..5] = max).
__global__ void k_level_bbox(const uint64_t* __restrict__ ukeys, int64_t V, int32_t* __restrict__ box) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int64_t q[3];
    unpack_key(ukeys[v], q);
    for (int a = 0; a < 3; ++a) {
        atomicMin(box + a, (int32_t)q[a]);
        atomicMax(box + 3 + a, (int32_t)q[a]);
    }
}

__global__ void k_level_insert(const uint64_t* __restrict__ ukeys, int64_t V, uint64_t* __restrict__ slots,
                               uint32_t log2cap) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const uint64_t key = ukeys[v];
    const uint64_t val = (key << kIdxBits) | (uint64_t)v;
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t h = slot_of(key, log2cap);
    for (uint32_t it = 0; it <= mask; ++it) {
        const unsigned long long prev =
            atomicCAS((unsigned long long*)(slots + h), (unsigned long long)kEmpty, (unsigned long long)val);
        if (prev == (unsigned long long)kEmpty) return;
        h = (h + 1u) & mask;
    }
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static int grid_of(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

size_t build_level_scratch_bytes(int64_t n) {
    size_t a = 0, b = 0, c = 0;
    const int N = (int)(n > 0 ? n : 1);
    hipcub::DeviceRadixSort::SortPairs(nullptr, a, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                       (int32_t*)nullptr, N, 0, 3 * kKeyBits);
    hipcub::DeviceRunLengthEncode::Encode(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                          (int32_t*)nullptr, N);
    hipcub::DeviceScan::ExclusiveSum(nullptr, c, (int32_t*)nullptr, (int32_t*)nullptr, N);
    return std::max(a, std::max(b, c)) + 256;
}

// Scratch layout (n entries each): keys_in, keys_out (u64), idx_in, idx_out,
// counts, offsets (i32), unique keys (u64), and `d_sort_tmp` for hipcub.
vg_status build_level(vg_context* ctx, const double* d_xyz, const double* d_cov, int64_t n, double r,
                      const double origin[3], Level* out, uint64_t* d_scratch_keys, int32_t* d_scratch_idx,
                      void* d_sort_tmp, size_t sort_tmp_bytes, int32_t* d_flag) {
    hipStream_t st = ctx->stream;
    out->r = r;
    for (int a = 0; a < 3; ++a) out->K0[a] = (int64_t)llround(origin[a] / r);
    out->V = 0;
    if (n > 0) {
        uint64_t* keys_in = d_scratch_keys;
        uint64_t* keys_out = d_scratch_keys + n;
        uint64_t* ukeys = d_scratch_keys + 2 * n;
        int32_t* idx_in = d_scratch_idx;
        int32_t* idx_out = d_scratch_idx + n;
        int32_t* counts = d_scratch_idx + 2 * n;
        int32_t* offsets = d_scratch_idx + 3 * n;
        int32_t* nruns = d_scratch_idx + 4 * n;
        VG_HIP(hipMemsetAsync(d_flag, 0, sizeof(int32_t), st));
        k_level_keys<<<grid_of(n), 256, 0, st>>>(d_xyz, n, r, out->K0[0], out->K0[1], out->K0[2], keys_in, idx_in,
                                                 d_flag);
        VG_HIP(hipGetLastError());
        int32_t h_flag = 0;
        VG_HIP(hipMemcpyAsync(&h_flag, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        if (h_flag) {
            set_error("voxel key outside the packable range (|q - q_origin| >= 8192 voxels on an axis)");
            return VG_ERR_KEY_RANGE;
        }
        size_t tb = sort_tmp_bytes;
        VG_HIP(hipcub::DeviceRadixSort::SortPairs(d_sort_tmp, tb, keys_in, keys_out, idx_in, idx_out, (int)n, 0,
                                                  3 * kKeyBits, st));
        tb = sort_tmp_bytes;
        VG_HIP(hipcub::DeviceRunLengthEncode::Encode(d_sort_tmp, tb, keys_out, ukeys, counts, nruns, (int)n, st));
        int32_t V = 0;
        VG_HIP(hipMemcpyAsync(&V, nruns, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        if (V > kMaxVoxels) {
            set_error("too many voxels in one level");
            return VG_ERR_CAPACITY;
        }
        tb = sort_tmp_bytes;
        VG_HIP(hipcub::DeviceScan::ExclusiveSum(d_sort_tmp, tb, counts, offsets, V, st));
        out->V = V;
        VG_HIP(hipMalloc(&out->rec32, sizeof(float) * kRec32 * (size_t)V));
        VG_HIP(hipMalloc(&out->recN, sizeof(float) * kRecN * (size_t)V));
        VG_HIP(hipMalloc(&out->rec64, sizeof(double) * kRec64 * (size_t)V));
        VG_HIP(hipMalloc(&out->keys, sizeof(uint64_t) * (size_t)V));
        VG_HIP(hipMalloc(&out->counts, sizeof(int32_t) * (size_t)V));
        k_level_stats<<<grid_of(V), 256, 0, st>>>(d_xyz, d_cov, ukeys, counts, offsets, idx_out, V, r, out->K0[0],
                                                  out->K0[1], out->K0[2], out->rec32, out->recN, out->rec64,
                                                  out->keys, out->counts);
        VG_HIP(hipGetLastError());
    }
    // capacity: power of two >= 4 V (load factor <= 1/4, so most misses end at
    // the first slot), at least 64 slots
    uint32_t lg = 6;
    while ((1ull << lg) < 4ull * (uint64_t)out->V) ++lg;
    out->log2cap = lg;
    const int64_t cap = 1ll << lg;
    VG_HIP(hipMalloc(&out->slots, sizeof(uint64_t) * (size_t)cap));
    k_fill_u64<<<grid_of(cap), 256, 0, st>>>(out->slots, cap, kEmpty);
    VG_HIP(hipGetLastError());
    if (out->V > 0) {
        k_level_insert<<<grid_of(out->V), 256, 0, st>>>(out->keys, out->V, out->slots, lg);
        VG_HIP(hipGetLastError());
        int32_t h_box[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
        VG_HIP(hipMemcpyAsync(d_flag, h_box, sizeof(h_box), hipMemcpyHostToDevice, st));
        k_level_bbox<<<grid_of(out->V), 256, 0, st>>>(out->keys, out->V, d_flag);
        VG_HIP(hipGetLastError());
        VG_HIP(hipMemcpyAsync(h_box, d_flag, sizeof(h_box), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        for (int a = 0; a < 3; ++a) {
            out->kmin[a] = h_box[a];
            out->kmax[a] = h_box[3 + a];
        }
    }
    VG_HIP(hipStreamSynchronize(st));
    return VG_OK;
}

vg_status export_level(vg_context* ctx, const Level& lv, int64_t* keys, double* means, double* covs,
                       int64_t* counts) {
    hipStream_t st = ctx->stream;
    const int64_t V = lv.V;
    if (V == 0) return VG_OK;
    std::vector<uint64_t> k((size_t)V);
    std::vector<int32_t> c((size_t)V);
    std::vector<double> r((size_t)V * kRec64);
    VG_HIP(hipMemcpyAsync(k.data(), lv.keys, sizeof(uint64_t) * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipMemcpyAsync(c.data(), lv.counts, sizeof(int32_t) * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipMemcpyAsync(r.data(), lv.rec64, sizeof(double) * kRec64 * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    for (int64_t v = 0; v < V; ++v) {
        int64_t q[3];
        unpack_key(k[v], q);
        if (keys)
            for (int a = 0; a < 3; ++a) keys[3 * v + a] = q[a] + lv.K0[a];
        if (means)
            for (int a = 0; a < 3; ++a) means[3 * v + a] = r[kRec64 * v + a];
        if (covs)
            for (int a = 0; a < 6; ++a) covs[6 * v + a] = r[kRec64 * v + 3 + a];
        if (counts) counts[v] = c[v];
    }
    return VG_OK;
}

void free_level(Level* lv) {
    if (lv->slots) (void)hipFree(lv->slots);
    if (lv->rec32) (void)hipFree(lv->rec32);
    if (lv->recN) (void)hipFree(lv->recN);
    if (lv->rec64) (void)hipFree(lv->rec64);
    if (lv->keys) (void)hipFree(lv->keys);
    if (lv->counts) (void)hipFree(lv->counts);
    *lv = Level{};
}

// ---------------------------------------------------------------- source clouds

__device__ __forceinline__ uint64_t spread21(uint64_t v) {
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Morton code of 0.25 m cells around the source origin (21 bits per axis).
__global__ void k_morton(const double* __restrict__ xyz, int64_t n, double ox, double oy, double oz,
                         uint64_t* __restrict__ codes, int32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double o[3] = {ox, oy, oz};
    uint64_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double c = floor((xyz[3 * i + a] - o[a]) * 4.0) + 1048576.0;
        c = fmin(fmax(c, 0.0), 2097151.0);
        q[a] = (uint64_t)c;
    }
    codes[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
    idx[i] = (int32_t)i;
}

__global__ void k_layout(const double* __restrict__ xyz, const double* __restrict__ cov,
                         const double* __restrict__ nrm, const int32_t* __restrict__ sorted_idx, int64_t n,
                         int64_t n_pad, float* __restrict__ dxyz, float* __restrict__ cov32, float* __restrict__ nrm32,
                         double* __restrict__ anchor, float* __restrict__ axyz, double* __restrict__ xyz64,
                         double* __restrict__ cov64, double* __restrict__ nrm64, int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    const int64_t c = i / kChunk;
    const double an[3] = {anchor[3 * c + 0], anchor[3 * c + 1], anchor[3 * c + 2]};
    if (i < n) {
        const int64_t s = sorted_idx[i];
        perm[i] = (int32_t)s;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double x = xyz[3 * s + q];
            dxyz[q * n_pad + i] = (float)(x - an[q]);
            axyz[q * n_pad + i] = (float)x;
            xyz64[q * n_pad + i] = x;
            if (nrm) {
                nrm32[q * n_pad + i] = (float)nrm[3 * s + q];
                nrm64[q * n_pad + i] = nrm[3 * s + q];
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            cov32[k * n_pad + i] = (float)cov[6 * s + k];
            cov64[k * n_pad + i] = cov[6 * s + k];
        }
    } else {
        perm[i] = -1;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            dxyz[q * n_pad + i] = 0.f;
            axyz[q * n_pad + i] = 0.f;
            xyz64[q * n_pad + i] = 0.0;
            if (nrm) {
                nrm32[q * n_pad + i] = 0.f;
                nrm64[q * n_pad + i] = 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            cov32[k * n_pad + i] = 0.f;
            cov64[k * n_pad + i] = 0.0;
        }
    }
}

// Anchor of each 64-point chunk: the centroid of its points (keeps the FP32
// offsets, and so their rounding, as small as the chunk allows).
__global__ void k_anchors(const double* __restrict__ xyz, const int32_t* __restrict__ sorted_idx, int64_t n,
                          int64_t n_chunks, double* __restrict__ anchor) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    const int64_t i0 = c * kChunk;
    const int64_t i1 = (i0 + kChunk < n) ? i0 + kChunk : n;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < i1; ++i) {
        const int64_t p = sorted_idx[i];
        s[0] += xyz[3 * p + 0];
        s[1] += xyz[3 * p + 1];
        s[2] += xyz[3 * p + 2];
    }
    const double inv = 1.0 / (double)(i1 - i0);
    anchor[3 * c + 0] = s[0] * inv;
    anchor[3 * c + 1] = s[1] * inv;
    anchor[3 * c + 2] = s[2] * inv;
}

vg_status layout_source(vg_context* ctx, vg_source* s, const double* d_xyz, const double* d_cov,
                        const double* d_nrm) {
    hipStream_t st = ctx->stream;
    const int64_t n = s->n, n_pad = s->n_pad;
    if (n == 0) return VG_OK;
    uint64_t *codes = nullptr, *codes2 = nullptr;
    int32_t *idx = nullptr, *idx2 = nullptr;
    void* tmp = nullptr;
    size_t tb = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                       (int32_t*)nullptr, (int)n, 0, 63);
    vg_status rc = VG_OK;
    hipError_t e = hipSuccess;
    do {
        if ((e = hipMalloc(&codes, 8 * n)) != hipSuccess) break;
        if ((e = hipMalloc(&codes2, 8 * n)) != hipSuccess) break;
        if ((e = hipMalloc(&idx, 4 * n)) != hipSuccess) break;
        if ((e = hipMalloc(&idx2, 4 * n)) != hipSuccess) break;
        if ((e = hipMalloc(&tmp, tb + 256)) != hipSuccess) break;
        k_morton<<<grid_of(n), 256, 0, st>>>(d_xyz, n, s->origin[0], s->origin[1], s->origin[2], codes, idx);
        if ((e = hipGetLastError()) != hipSuccess) break;
        size_t tb2 = tb + 256;
        if ((e = hipcub::DeviceRadixSort::SortPairs(tmp, tb2, codes, codes2, idx, idx2, (int)n, 0, 63, st)) !=
            hipSuccess)
            break;
        k_anchors<<<grid_of(s->n_chunks), 256, 0, st>>>(d_xyz, idx2, n, s->n_chunks, s->anchor);
        if ((e = hipGetLastError()) != hipSuccess) break;
        k_layout<<<grid_of(n_pad), 256, 0, st>>>(d_xyz, d_cov, d_nrm, idx2, n, n_pad, s->dxyz, s->cov, s->nrm,
                                                 s->anchor, s->axyz, s->xyz64, s->cov64, s->nrm64, s->perm);
        if ((e = hipGetLastError()) != hipSuccess) break;
        e = hipStreamSynchronize(st);
    } while (0);
    if (e != hipSuccess) rc = hip_fail(e, "source layout");
    if (codes) (void)hipFree(codes);
    if (codes2) (void)hipFree(codes2);
    if (idx) (void)hipFree(idx);
    if (idx2) (void)hipFree(idx2);
    if (tmp) (void)hipFree(tmp);
    return rc;
}

template <typename S>
__global__ void k_set_points(const S* __restrict__ in, const int32_t* __restrict__ perm,
                             const double* __restrict__ anchor, int64_t n, int64_t n_pad, float* __restrict__ dxyz,
                             float* __restrict__ axyz, double* __restrict__ xyz64) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t s = perm[i];
    const int64_t c = i / kChunk;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double x = (double)in[3 * s + q];
        dxyz[q * n_pad + i] = (float)(x - anchor[3 * c + q]);
        axyz[q * n_pad + i] = (float)x;
        xyz64[q * n_pad + i] = x;
    }
}

vg_status set_source_points(vg_context* ctx, vg_source* s, const void* d_xyz, int dtype) {
    if (s->n == 0) return VG_OK;
    if (dtype == 0)
        k_set_points<float><<<grid_of(s->n), 256, 0, ctx->stream>>>((const float*)d_xyz, s->perm, s->anchor, s->n,
                                                                    s->n_pad, s->dxyz, s->axyz, s->xyz64);
    else
        k_set_points<double><<<grid_of(s->n), 256, 0, ctx->stream>>>((const double*)d_xyz, s->perm, s->anchor, s->n,
                                                                     s->n_pad, s->dxyz, s->axyz, s->xyz64);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

}  // namespace vg
