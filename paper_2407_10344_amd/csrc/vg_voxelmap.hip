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
#include <vector>

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

// Per-voxel statistics of voxel v (canonical = ascending-key order): FP64 sums
// of its points in ascending point order, then the average; records are
// written at position pos[v] (block order).
__global__ void k_level_stats(const double* __restrict__ xyz, const double* __restrict__ cov,
                              const uint64_t* __restrict__ ukeys, const int32_t* __restrict__ counts,
                              const int32_t* __restrict__ offsets, const int32_t* __restrict__ sorted_idx,
                              const int32_t* __restrict__ pos, int64_t V, double r, int64_t K0x, int64_t K0y,
                              int64_t K0z, float* __restrict__ rec32, float* __restrict__ recN,
                              double* __restrict__ rec64) {
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
    int64_t q[3];
    unpack_key(ukeys[v], q);
    q[0] += K0x;
    q[1] += K0y;
    q[2] += K0z;
    const int64_t w = pos[v];
    double* r64 = rec64 + kRec64 * w;
    float* r32 = rec32 + kRec32 * w;
    double* r32c = reinterpret_cast<double*>(r32 + 4);   // 8-byte aligned: records are 64 B
    float* rN = recN + kRecN * w;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double centre = (double)q[a] * r + 0.5 * r;
        r64[a] = m[a];
        r32[a] = (float)(m[a] - centre);
        rN[a] = (float)m[a];
    }
    r32[3] = (float)cnt;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        r64[3 + k] = m[3 + k];
        r32c[k] = m[3 + k];                             // covariance, FP64
        rN[3 + k] = (float)m[3 + k];
    }
    r64[9] = 0.0;
    rN[9] = 0.f;
    rN[10] = 0.f;
    rN[11] = 0.f;
}

// Block-order sort key of voxel v: (block key << 6) | Morton index inside the block.
__global__ void k_block_codes(const uint64_t* __restrict__ ukeys, int64_t V, uint64_t* __restrict__ codes,
                              int32_t* __restrict__ idx) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int64_t q[3];
    unpack_key(ukeys[v], q);
    const uint64_t ux = (uint64_t)(q[0] + kKeyBias), uy = (uint64_t)(q[1] + kKeyBias), uz = (uint64_t)(q[2] + kKeyBias);
    codes[v] = (block_key(ux, uy, uz) << 6) | block_local(ux, uy, uz);
    idx[v] = (int32_t)v;
}

// pos[canonical index] = record position, and the block key of every record.
__global__ void k_block_scatter(const uint64_t* __restrict__ codes_sorted, const int32_t* __restrict__ idx_sorted,
                                int64_t V, int32_t* __restrict__ pos, uint64_t* __restrict__ bkeys) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= V) return;
    pos[idx_sorted[m]] = (int32_t)m;
    bkeys[m] = codes_sorted[m] >> 6;
}

// One thread per occupied block: occupancy mask of its records, then insertion
// of (block key | first record, mask) into the block table.
__global__ void k_block_insert(const uint64_t* __restrict__ ublocks, const int32_t* __restrict__ bcounts,
                               const int32_t* __restrict__ boffsets, const uint64_t* __restrict__ codes_sorted,
                               int64_t NB, uint64_t* __restrict__ slots, uint32_t log2cap) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= NB) return;
    const int32_t base = boffsets[b], cnt = bcounts[b];
    uint64_t occ = 0;
    for (int32_t m = base; m < base + cnt; ++m) occ |= 1ull << (codes_sorted[m] & 63);
    const uint64_t key = ublocks[b];
    const uint64_t word = (key << kBaseBits) | (uint64_t)base;
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t h = slot_of(key, log2cap);
    for (uint32_t it = 0; it <= mask; ++it) {
        const unsigned long long prev = atomicCAS((unsigned long long*)(slots + 2 * (uint64_t)h),
                                                  (unsigned long long)kEmpty, (unsigned long long)word);
        if (prev == (unsigned long long)kEmpty) {
            slots[2 * (uint64_t)h + 1] = occ;
            return;
        }
        h = (h + 1u) & mask;
    }
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

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static int grid_of(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

namespace {
// Device scratch owned by one build call.
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * (count ? count : 1));
        if (e == hipSuccess) ptrs.push_back(q);
        *p = (T*)q;
        return e;
    }
};
}  // namespace

vg_status build_level(vg_context* ctx, const double* d_xyz, const double* d_cov, int64_t n, double r,
                      const double origin[3], Level* out) {
    hipStream_t st = ctx->stream;
    out->r = r;
    for (int a = 0; a < 3; ++a) out->K0[a] = (int64_t)llround(origin[a] / r);
    out->V = 0;
    out->n_blocks = 0;
    Scratch sc;
    int32_t* d_small = nullptr;   // flag, run counts, bbox
    VG_HIP(sc.get(&d_small, 64));
    if (n > 0) {
        uint64_t *keys_in, *keys_out, *ukeys, *codes, *codes_sorted, *bkeys, *ublocks;
        int32_t *idx_in, *idx_out, *counts, *offsets, *vidx, *vidx_sorted, *pos, *bcounts, *boffsets;
        VG_HIP(sc.get(&keys_in, n));
        VG_HIP(sc.get(&keys_out, n));
        VG_HIP(sc.get(&idx_in, n));
        VG_HIP(sc.get(&idx_out, n));
        VG_HIP(sc.get(&counts, n));
        VG_HIP(sc.get(&offsets, n));
        size_t tmp_bytes = 0, b2 = 0, b3 = 0;
        (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys_in, keys_out, idx_in, idx_out, (int)n, 0,
                                                 3 * kKeyBits);
        (void)hipcub::DeviceRunLengthEncode::Encode(nullptr, b2, keys_out, keys_in, counts, d_small, (int)n);
        (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b3, counts, offsets, (int)n);
        tmp_bytes = std::max(tmp_bytes, std::max(b2, b3)) + 256;
        void* tmp = nullptr;
        VG_HIP(sc.get((char**)&tmp, tmp_bytes));
        // 1. keys of every point, stable sort by key, runs = voxels
        VG_HIP(hipMemsetAsync(d_small, 0, sizeof(int32_t), st));
        k_level_keys<<<grid_of(n), 256, 0, st>>>(d_xyz, n, r, out->K0[0], out->K0[1], out->K0[2], keys_in, idx_in,
                                                 d_small);
        VG_HIP(hipGetLastError());
        int32_t h_flag = 0;
        VG_HIP(hipMemcpyAsync(&h_flag, d_small, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        if (h_flag) {
            set_error("voxel key outside the packable range (|q - q_origin| >= 8192 voxels on an axis)");
            return VG_ERR_KEY_RANGE;
        }
        size_t tb = tmp_bytes;
        VG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys_in, keys_out, idx_in, idx_out, (int)n, 0,
                                                  3 * kKeyBits, st));
        VG_HIP(sc.get(&ukeys, n));
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, keys_out, ukeys, counts, d_small + 1, (int)n, st));
        int32_t V = 0;
        VG_HIP(hipMemcpyAsync(&V, d_small + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        if (V > kMaxVoxels) {
            set_error("too many voxels in one level");
            return VG_ERR_CAPACITY;
        }
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, counts, offsets, V, st));
        out->V = V;
        // 2. block order of the voxels and their record positions
        VG_HIP(sc.get(&codes, V));
        VG_HIP(sc.get(&codes_sorted, V));
        VG_HIP(sc.get(&vidx, V));
        VG_HIP(sc.get(&vidx_sorted, V));
        VG_HIP(sc.get(&bkeys, V));
        VG_HIP(sc.get(&ublocks, V));
        VG_HIP(sc.get(&bcounts, V));
        VG_HIP(sc.get(&boffsets, V));
        VG_HIP(hipMalloc(&out->lex2rec, sizeof(int32_t) * (size_t)V));
        pos = out->lex2rec;
        k_block_codes<<<grid_of(V), 256, 0, st>>>(ukeys, V, codes, vidx);
        VG_HIP(hipGetLastError());
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, codes, codes_sorted, vidx, vidx_sorted, V, 0,
                                                  3 * kBlockBits + 6, st));
        k_block_scatter<<<grid_of(V), 256, 0, st>>>(codes_sorted, vidx_sorted, V, pos, bkeys);
        VG_HIP(hipGetLastError());
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, bkeys, ublocks, bcounts, d_small + 2, V, st));
        int32_t NB = 0;
        VG_HIP(hipMemcpyAsync(&NB, d_small + 2, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, bcounts, boffsets, NB, st));
        out->n_blocks = NB;
        // 3. records in block order
        VG_HIP(hipMalloc(&out->rec32, sizeof(float) * kRec32 * (size_t)V));
        VG_HIP(hipMalloc(&out->recN, sizeof(float) * kRecN * (size_t)V));
        VG_HIP(hipMalloc(&out->rec64, sizeof(double) * kRec64 * (size_t)V));
        VG_HIP(hipMalloc(&out->keys, sizeof(uint64_t) * (size_t)V));
        VG_HIP(hipMalloc(&out->counts, sizeof(int32_t) * (size_t)V));
        k_level_stats<<<grid_of(V), 256, 0, st>>>(d_xyz, d_cov, ukeys, counts, offsets, idx_out, pos, V, r,
                                                  out->K0[0], out->K0[1], out->K0[2], out->rec32, out->recN,
                                                  out->rec64);
        VG_HIP(hipGetLastError());
        VG_HIP(hipMemcpyAsync(out->keys, ukeys, sizeof(uint64_t) * V, hipMemcpyDeviceToDevice, st));
        VG_HIP(hipMemcpyAsync(out->counts, counts, sizeof(int32_t) * V, hipMemcpyDeviceToDevice, st));
        // 4. block table: power of two >= 4 x blocks (load factor <= 1/4)
        uint32_t lg = 6;
        while ((1ull << lg) < 4ull * (uint64_t)NB) ++lg;
        out->log2cap = lg;
        const int64_t cap = 1ll << lg;
        VG_HIP(hipMalloc(&out->slots, sizeof(uint64_t) * 2 * (size_t)cap));
        k_fill_u64<<<grid_of(2 * cap), 256, 0, st>>>(out->slots, 2 * cap, kEmpty);
        VG_HIP(hipGetLastError());
        k_block_insert<<<grid_of(NB), 256, 0, st>>>(ublocks, bcounts, boffsets, codes_sorted, NB, out->slots, lg);
        VG_HIP(hipGetLastError());
        // 5. key bounding box
        int32_t h_box[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
        VG_HIP(hipMemcpyAsync(d_small + 8, h_box, sizeof(h_box), hipMemcpyHostToDevice, st));
        k_level_bbox<<<grid_of(V), 256, 0, st>>>(ukeys, V, d_small + 8);
        VG_HIP(hipGetLastError());
        VG_HIP(hipMemcpyAsync(h_box, d_small + 8, sizeof(h_box), hipMemcpyDeviceToHost, st));
        VG_HIP(hipStreamSynchronize(st));
        for (int a = 0; a < 3; ++a) {
            out->kmin[a] = h_box[a];
            out->kmax[a] = h_box[3 + a];
        }
    } else {
        out->log2cap = 6;
        VG_HIP(hipMalloc(&out->slots, sizeof(uint64_t) * 2 * 64));
        k_fill_u64<<<1, 128, 0, st>>>(out->slots, 128, kEmpty);
        VG_HIP(hipGetLastError());
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
    std::vector<int32_t> c((size_t)V), l2r((size_t)V);
    std::vector<double> r((size_t)V * kRec64);
    VG_HIP(hipMemcpyAsync(k.data(), lv.keys, sizeof(uint64_t) * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipMemcpyAsync(c.data(), lv.counts, sizeof(int32_t) * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipMemcpyAsync(l2r.data(), lv.lex2rec, sizeof(int32_t) * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipMemcpyAsync(r.data(), lv.rec64, sizeof(double) * kRec64 * V, hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    for (int64_t v = 0; v < V; ++v) {
        int64_t q[3];
        unpack_key(k[v], q);
        const int64_t w = l2r[v];
        if (keys)
            for (int a = 0; a < 3; ++a) keys[3 * v + a] = q[a] + lv.K0[a];
        if (means)
            for (int a = 0; a < 3; ++a) means[3 * v + a] = r[kRec64 * w + a];
        if (covs)
            for (int a = 0; a < 6; ++a) covs[6 * v + a] = r[kRec64 * w + 3 + a];
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
    if (lv->lex2rec) (void)hipFree(lv->lex2rec);
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

// FP32 value >= x (round up).
__device__ __forceinline__ float f32_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

// Per chunk, from the FP32 offsets the kernels read: a ball around the anchor
// (radius bounds every point's distance) and an axis-aligned box in the source
// frame (centre offset from the anchor, half extents bounding every point).
__global__ void k_chunk_bounds(const float* __restrict__ dxyz, int64_t n, int64_t n_pad, int64_t n_chunks,
                               float* __restrict__ cb) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    const int64_t i0 = c * kChunk;
    const int64_t i1 = (i0 + kChunk < n) ? i0 + kChunk : n;
    double m = 0.0, lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0; i < i1; ++i) {
        const double x[3] = {dxyz[i], dxyz[n_pad + i], dxyz[2 * n_pad + i]};
        m = fmax(m, x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        for (int a = 0; a < 3; ++a) {
            lo[a] = (i == i0) ? x[a] : fmin(lo[a], x[a]);
            hi[a] = (i == i0) ? x[a] : fmax(hi[a], x[a]);
        }
    }
    float* o = cb + 8 * c;
    for (int a = 0; a < 3; ++a) {
        const float ctr = (float)(0.5 * (lo[a] + hi[a]));
        o[a] = ctr;
        o[4 + a] = f32_up(fmax(hi[a] - (double)ctr, (double)ctr - lo[a]));
    }
    o[3] = f32_up(sqrt(m));
    o[7] = 0.f;
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
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
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
        k_chunk_bounds<<<grid_of(s->n_chunks), 256, 0, st>>>(s->dxyz, n, n_pad, s->n_chunks, s->cbound);
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
    // the offsets moved: so do the chunk bounds
    k_chunk_bounds<<<grid_of(s->n_chunks), 256, 0, ctx->stream>>>(s->dxyz, s->n, s->n_pad, s->n_chunks, s->cbound);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

}  // namespace vg
