// Device helpers shared by the VGICP kernels: key packing, hash probing and
// small symmetric 3x3 algebra.
#pragma once

#include "vg_internal.h"

namespace vg {

// Global-address-space view of a device pointer read from a descriptor in
// memory: loads through it compile to global_load (not flat_load, which also
// waits on the LDS counter).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gbl(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// Native vector types for 16-byte loads through global pointers.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x3 __attribute__((ext_vector_type(3)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Relative voxel key (|k| < 8192 per axis) packed into 42 bits; x is the most
// significant field, so ascending packed keys are ascending lexicographic keys.
__host__ __device__ __forceinline__ bool key_in_range(int64_t k) {
    return k >= -kKeyBias && k < kKeyBias;
}

__host__ __device__ __forceinline__ uint64_t pack_key(int64_t kx, int64_t ky, int64_t kz) {
    return ((uint64_t)(kx + kKeyBias) << (2 * kKeyBits)) | ((uint64_t)(ky + kKeyBias) << kKeyBits) |
           (uint64_t)(kz + kKeyBias);
}

__host__ __device__ __forceinline__ void unpack_key(uint64_t p, int64_t k[3]) {
    const uint64_t m = (1ull << kKeyBits) - 1;
    k[0] = (int64_t)((p >> (2 * kKeyBits)) & m) - kKeyBias;
    k[1] = (int64_t)((p >> kKeyBits) & m) - kKeyBias;
    k[2] = (int64_t)(p & m) - kKeyBias;
}

// Slot of a block: Fibonacci hashing (the top bits of one 32-bit product with
// the golden-ratio constant) of the block key (bx << 24 | by << 12 | bz, 12
// bits per coordinate, 36 bits) folded into one word by XOR of its two words,
// which the lookup forms anyway for the key compare.
__host__ __device__ __forceinline__ uint32_t slot_of_words(uint32_t lo, uint32_t hi, uint32_t log2cap) {
    return ((lo ^ hi) * 0x9E3779B1u) >> (32u - log2cap);
}
__host__ __device__ __forceinline__ uint32_t slot_of(uint64_t bk, uint32_t log2cap) {
    return slot_of_words((uint32_t)bk, (uint32_t)(bk >> 32), log2cap);
}

// Sparse-block voxel lookup.  Voxels are grouped in 4 x 4 x 4 blocks; a hash
// table (open addressing, linear probing, load factor <= 1/4) maps each
// occupied block to one 16-byte entry: (block key << 28 | index of the block's
// first record) and a 64-bit occupancy mask.  Records are stored block by
// block, x fastest inside a block (bit x + 4 y + 16 z), so a voxel's record
// index is first + popcount(mask below its bit).  Neighbouring points share
// block entries and read neighbouring records.
__host__ __device__ __forceinline__ uint32_t block_local(uint64_t ux, uint64_t uy, uint64_t uz) {
    return (uint32_t)((ux & 3) | ((uy & 3) << 2) | ((uz & 3) << 4));
}

__host__ __device__ __forceinline__ uint64_t block_key(uint64_t ux, uint64_t uy, uint64_t uz) {
    return ((ux >> kBlockShift) << (2 * kBlockBits)) | ((uy >> kBlockShift) << kBlockBits) | (uz >> kBlockShift);
}

// Load of a T at a 32-bit byte offset from a base pointer.  With a uniform
// base this compiles to a global load with the base in scalar registers and
// only the 32-bit offset in a vector register (no 64-bit address arithmetic
// per lane).
template <typename T>
__device__ __forceinline__ T load_off(const void* base, uint32_t byte_off) {
    return *gbl(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint64_t)byte_off));
}

// (a & M) | (b & ~M) for a small constant mask M, as one v_bfi_b32
template <uint32_t M>
__device__ __forceinline__ uint32_t bfi_low(uint32_t a, uint32_t b) {
    static_assert(M <= 64, "an inline constant");
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "n"(M), "v"(a), "v"(b));
    return r;
}

// Record index of the voxel with biased key (ux, uy, uz) = relative key + 8192
// (each in [0, 16383]), or -1, in two halves so a caller can do other work
// while the first table load is in flight: lookup_issue forms the block key,
// slot and bit and issues the load; lookup_finish takes the result.  The first
// table entry decides almost every lookup (load factor <= 1/4): it is either
// the block, or empty, or (rarely) another block, and only then is the chain
// walked.  The occupancy test and the popcount below the voxel's bit work on
// the 64-bit mask as a whole.
struct BlockProbe {
    u64x2 e;           // the table entry (first slot until the chain is walked)
    uint64_t bk;       // block key
    uint32_t h;        // slot
    uint32_t nlocal;   // 63 - bit of the voxel in its block's mask (in bits 0..5)
};
__device__ __forceinline__ void lookup_issue(const uint64_t* __restrict__ slots, uint32_t log2cap, uint32_t ux,
                                             uint32_t uy, uint32_t uz, BlockProbe& p) {
    const uint32_t bx = ux >> kBlockShift, by = uy >> kBlockShift, bz = uz >> kBlockShift;
    const uint32_t klo = (bx << (2 * kBlockBits)) | (by << kBlockBits) | bz, khi = bx >> (32 - 2 * kBlockBits);
    p.bk = ((uint64_t)khi << 32) | klo;
    p.h = slot_of_words(klo, khi, log2cap);
    p.e = load_off<u64x2>(slots, p.h << 4);
    // bit of the voxel in the mask: x + 4 y + 16 z of its position in the block
    // (two bit-field inserts), complemented in bits 0..5; the bits above are
    // left over from z, and the 64-bit shift below reads only bits 0..5
    p.nlocal = bfi_low<15u>(bfi_low<3u>(ux, uy << 2), uz << 4) ^ 63u;
}
__device__ __forceinline__ int32_t lookup_finish(const uint64_t* __restrict__ slots, uint32_t log2cap,
                                                 BlockProbe& p) {
    bool same = (p.e.x >> kBaseBits) == p.bk;
    if (!same && p.e.x != kEmpty) {
        // another block in the first slot: walk the chain (linear probing)
        const uint32_t mask = (1u << log2cap) - 1u;
        uint32_t h = p.h;
        for (uint32_t it = 0; it < mask; ++it) {
            h = (h + 1u) & mask;
            p.e = load_off<u64x2>(slots, h << 4);
            same = (p.e.x >> kBaseBits) == p.bk;
            if (same || p.e.x == kEmpty) break;
        }
    }
    // the mask shifted left by 63 - bit: the voxel's bit becomes the sign bit,
    // and the bits left are those at and below it, so their count is the
    // voxel's rank among the block's occupied voxels plus one.  An empty entry
    // never holds the block (a valid entry word is never all ones).
    const uint64_t t = p.e.y << (p.nlocal & 63u);
    const bool occupied = (int32_t)(uint32_t)(t >> 32) < 0;
    const uint32_t cnt = ((uint32_t)p.e.x & (uint32_t)kBaseMask) + (uint32_t)__popc((uint32_t)t) +
                         (uint32_t)__popc((uint32_t)(t >> 32));
    return (same && p.e.x != kEmpty && occupied) ? (int32_t)(cnt - 1u) : -1;
}
__device__ __forceinline__ int32_t lookup_u(const uint64_t* __restrict__ slots, uint32_t log2cap, uint32_t ux,
                                            uint32_t uy, uint32_t uz) {
    BlockProbe p;
    lookup_issue(slots, log2cap, ux, uy, uz, p);
    return lookup_finish(slots, log2cap, p);
}

// The same for a relative key (kx, ky, kz) (each in [-8192, 8191]).
__device__ __forceinline__ int32_t lookup(const uint64_t* __restrict__ slots, uint32_t log2cap, int32_t kx,
                                          int32_t ky, int32_t kz) {
    return lookup_u(slots, log2cap, (uint32_t)(kx + kKeyBias), (uint32_t)(ky + kKeyBias), (uint32_t)(kz + kKeyBias));
}

// Buffer resource over `bytes` bytes at p (raw buffer, no swizzle): loads
// through it take a scalar base plus a 32-bit offset and return 0 beyond the
// end instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float rsrc_load_f32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// 1/x without the correctly rounded division sequence: hardware reciprocal
// refined by Newton steps (two for FP64, each doubling the correct bits).
__device__ __forceinline__ float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// floor(x) as an int32 in one instruction (v_cvt_flr_i32_f32; equal to
// (int32_t)floorf(x) for finite x in the int32 range, which holds for every
// chunk-relative key position the kernels form).
__device__ __forceinline__ int32_t floor_i32(float x) {
    int32_t r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Position of a point relative to its chunk anchor's coarse voxel corner, in
// FP32, with an explicit FMA order so every kernel that derives voxel keys
// from it gets identical bits.
__device__ __forceinline__ float chunk_pos32(float frac, float r0, float r1, float r2, float dx, float dy,
                                             float dz) {
    return fmaf(r2, dz, fmaf(r1, dy, fmaf(r0, dx, frac)));
}

// Per-chunk FP64 anchor transform for axis i: ya = (R a + t)_i (returned)
// split into the coarse voxel key (relative to the map origin, clamped far
// outside the key range) and the remainder inside that voxel.  Shared by every kernel that
// derives keys from chunk anchors so they agree bit for bit.
__device__ __forceinline__ double anchor_split(const double* __restrict__ P, const double a[3], int i, double r_top,
                                               double inv_r_top, int64_t K0_top, double* frac, int32_t* kb) {
    const double ya = fma(P[3 * i + 2], a[2], fma(P[3 * i + 1], a[1], P[3 * i] * a[0])) + P[9 + i];
    const double k = floor(ya * inv_r_top);
    *frac = ya - k * r_top;
    *kb = (int32_t)fmin(fmax(k - (double)K0_top, -1048576.0), 1048576.0);
    return ya;
}

// Inverse of a symmetric 3x3 matrix m = [a b c; b d e; c e f] via its adjugate.
// Entries ordered xx, xy, xz, yy, yz, zz.
template <typename T>
__device__ __forceinline__ void sym3_inverse(const T m[6], T w[6]) {
    const T a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
    const T A = d * f - e * e;
    const T B = c * e - b * f;
    const T C = b * e - c * d;
    const T D = a * f - c * c;
    const T E = b * c - a * e;
    const T Fv = a * d - b * b;
    const T det = a * A + b * B + c * C;
    const T s = recip(det);
    w[0] = A * s;
    w[1] = B * s;
    w[2] = C * s;
    w[3] = D * s;
    w[4] = E * s;
    w[5] = Fv * s;
}

// Inverse of a symmetric 3x3 matrix formed in FP64, rounded to FP32: the
// adjugate and determinant in FP64, 1/det by the hardware reciprocal and one
// Newton step (far below FP32 rounding).
__device__ __forceinline__ void sym3_inverse_f32(const double m[6], float w[6]) {
    const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
    const double A = d * f - e * e;
    const double B = c * e - b * f;
    const double C = b * e - c * d;
    const double det = a * A + b * B + c * C;
    double s = __builtin_amdgcn_rcp(det);
    s = fma(s, fma(-det, s, 1.0), s);
    w[0] = (float)(A * s);
    w[1] = (float)(B * s);
    w[2] = (float)(C * s);
    w[3] = (float)((a * f - c * c) * s);
    w[4] = (float)((b * c - a * e) * s);
    w[5] = (float)((a * d - b * b) * s);
}

// M = R C R^T + D for symmetric C and D (6 entries each) and row-major R, D
// added inside the last fused multiply-add of each entry.
template <typename T>
__device__ __forceinline__ void rotate_cov_add(const T R[9], const T c[6], const T D[6], T M[6]) {
    T RC[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T r0 = R[3 * i + 0], r1 = R[3 * i + 1], r2 = R[3 * i + 2];
        RC[3 * i + 0] = r0 * c[0] + r1 * c[1] + r2 * c[2];
        RC[3 * i + 1] = r0 * c[1] + r1 * c[3] + r2 * c[4];
        RC[3 * i + 2] = r0 * c[2] + r1 * c[4] + r2 * c[5];
    }
    M[0] = fma(RC[0], R[0], fma(RC[1], R[1], fma(RC[2], R[2], D[0])));
    M[1] = fma(RC[0], R[3], fma(RC[1], R[4], fma(RC[2], R[5], D[1])));
    M[2] = fma(RC[0], R[6], fma(RC[1], R[7], fma(RC[2], R[8], D[2])));
    M[3] = fma(RC[3], R[3], fma(RC[4], R[4], fma(RC[5], R[5], D[3])));
    M[4] = fma(RC[3], R[6], fma(RC[4], R[7], fma(RC[5], R[8], D[4])));
    M[5] = fma(RC[6], R[6], fma(RC[7], R[7], fma(RC[8], R[8], D[5])));
}

// S = R C R^T for symmetric C (6 entries) and row-major R; S returned as 6 entries.
template <typename T>
__device__ __forceinline__ void rotate_cov(const T R[9], const T c[6], T S[6]) {
    // RC = R * C (3x3)
    T RC[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T r0 = R[3 * i + 0], r1 = R[3 * i + 1], r2 = R[3 * i + 2];
        RC[3 * i + 0] = r0 * c[0] + r1 * c[1] + r2 * c[2];
        RC[3 * i + 1] = r0 * c[1] + r1 * c[3] + r2 * c[4];
        RC[3 * i + 2] = r0 * c[2] + r1 * c[4] + r2 * c[5];
    }
    S[0] = RC[0] * R[0] + RC[1] * R[1] + RC[2] * R[2];
    S[1] = RC[0] * R[3] + RC[1] * R[4] + RC[2] * R[5];
    S[2] = RC[0] * R[6] + RC[1] * R[7] + RC[2] * R[8];
    S[3] = RC[3] * R[3] + RC[4] * R[4] + RC[5] * R[5];
    S[4] = RC[3] * R[6] + RC[4] * R[7] + RC[5] * R[8];
    S[5] = RC[6] * R[6] + RC[7] * R[7] + RC[8] * R[8];
}

// y = W x for symmetric W (6 entries).
template <typename T>
__device__ __forceinline__ void sym3_mul(const T w[6], const T x[3], T y[3]) {
    y[0] = w[0] * x[0] + w[1] * x[1] + w[2] * x[2];
    y[1] = w[1] * x[0] + w[3] * x[1] + w[4] * x[2];
    y[2] = w[2] * x[0] + w[4] * x[1] + w[5] * x[2];
}

}  // namespace vg
