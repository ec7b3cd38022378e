// VGICP factor kernels for gfx950: transform + voxel-hash probe + fused-covariance
// residual + per-point Gauss-Newton terms, reduced per work tile, then per factor.
//
// GLIM Sec. III-C: e = sum_l sum_k d^T W d, d = mu~ - (R mu + t),
// W = (C~ + R C R^T)^-1 frozen at the linearization point, J = [R (mu)x, -R],
// H = sum J^T W J, b = sum J^T W d.
//
// Work decomposition.  A batch is a flat list of tiles (factor, run of 64-point
// chunks of its source).  A persistent grid pulls tiles from an atomic counter;
// every tile writes one partial row (28 terms + inlier counts) in FP64 to its own
// slot, and a second kernel sums each factor's rows in tile order, so results do
// not depend on which workgroup ran which tile.
//
// Frames.  The terms are accumulated in the target orientation: with
// z = R (mu - o_s) the per-point Jacobian is J = [(z)x, -I] Bd G where
// Bd = diag(R, R) and G = [[I, 0], [-(o_s)x, I]] are the same for every point of a
// factor, so the kernels sum H'' = sum [(z)x, -I]^T W [(z)x, -I] and
// b'' = [u x z; -u] (u = W d) and the reduction applies H = G^T Bd^T H'' Bd G,
// b = G^T Bd^T b'' once per factor in FP64.
//
// Precision modes.
//  kC32: positions are stored as FP32 offsets from per-chunk FP64 anchors.  Per
//        tile, each chunk's anchor is transformed in FP64 and split into an
//        integer coarse-voxel key plus an FP32 remainder, so every per-point
//        quantity (transformed position inside the coarse voxel, residual to a
//        voxel mean stored relative to its voxel centre, lever arm) is small and
//        FP32 keeps ~1e-7 m absolute accuracy anywhere in the map.  Lanes sum in
//        FP32 (optionally Kahan-compensated), everything above a lane in FP64.
//  kN32: absolute FP32 coordinates and FP32 sums everywhere.
//  kF64: absolute FP64 coordinates and arithmetic.
#include <type_traits>

#include "vg_device.h"

namespace vg {

template <int PREC>
struct PT {
    using T = float;
};
template <>
struct PT<kF64> {
    using T = double;
};

// Upper-triangular index of (i, j), i <= j, of a 6x6 matrix.
__host__ __device__ constexpr int tri(int i, int j) { return i * 6 - (i * (i - 1)) / 2 + (j - i); }

template <typename T, bool KAHAN, int N>
struct Acc {
    T s[N];
    T c[N];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < N; ++k) {
            s[k] = T(0);
            if constexpr (KAHAN) c[k] = T(0);
        }
    }
    __device__ __forceinline__ void add(int k, T v) {
        if constexpr (KAHAN) {
            const T y = v - c[k];
            const T t = s[k] + y;
            c[k] = (t - s[k]) - y;
            s[k] = t;
        } else {
            s[k] += v;
        }
    }
    // += a b + c d: two fused multiply-adds into the sum (one compensated add with Kahan)
    __device__ __forceinline__ void add2(int k, T a, T b, T c2, T d) {
        if constexpr (KAHAN) {
            add(k, fma(a, b, c2 * d));
        } else {
            s[k] = fma(c2, d, fma(a, b, s[k]));
        }
    }
    __device__ __forceinline__ T get(int k) const {
        if constexpr (KAHAN) return s[k] - c[k];
        else return s[k];
    }
    // the lane's sum with its compensation carried into FP64
    __device__ __forceinline__ double get64(int k) const {
        if constexpr (KAHAN) return (double)s[k] - (double)c[k];
        else return (double)s[k];
    }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// a + b after exchanging the upper half of a's lanes with the lower half of
// b's (stride 32: v_permlane32_swap; stride 16: v_permlane16_swap, which
// exchanges the odd 16-lane rows of a with the even rows of b).  Lanes whose
// stride bit is clear get a (own) + a (partner's), the others b (partner's) +
// b (own): one butterfly step of a wave sum that halves the values per lane.
template <int STRIDE>
__device__ __forceinline__ double swap_add(double a, double b) {
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const uint32_t alo = (uint32_t)ua, ahi = (uint32_t)(ua >> 32), blo = (uint32_t)ub, bhi = (uint32_t)(ub >> 32);
    uint32_t x0, x1, y0, y1;
    if constexpr (STRIDE == 32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        x0 = lo[0]; y0 = lo[1]; x1 = hi[0]; y1 = hi[1];
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        x0 = lo[0]; y0 = lo[1]; x1 = hi[0]; y1 = hi[1];
    }
    return __longlong_as_double((int64_t)(((uint64_t)x1 << 32) | x0)) +
           __longlong_as_double((int64_t)(((uint64_t)y1 << 32) | y0));
}

// Wave sum of 32 FP64 values per lane, transposed: each butterfly step keeps
// half of the values on each lane (the half selected by the lane's stride
// bit), so after five steps lanes 2k and 2k + 1 hold partial sums of value k
// over complementary halves of the wave, and the last step adds them.  Returns
// the sum of value lane / 2.  The order of the additions is fixed.
template <int O, int CNT>
__device__ __forceinline__ void xor_step(double (&v)[32], int lane) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
        const double send = up ? v[k] : v[k + CNT];
        const double keep = up ? v[k + CNT] : v[k];
        v[k] = keep + __shfl_xor(send, O, 64);
    }
}

__device__ __forceinline__ double wave_sum_transposed(double (&v)[32], int lane) {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = swap_add<32>(v[k], v[k + 16]);
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = swap_add<16>(v[k], v[k + 8]);
    xor_step<8, 4>(v, lane);
    xor_step<4, 2>(v, lane);
    xor_step<2, 1>(v, lane);
    return v[0] + __shfl_xor(v[0], 1, 64);
}

// Gauss-Newton terms of one (point, voxel) pair in the target orientation.
template <typename T, typename A>
__device__ __forceinline__ void add_lin_terms(A& acc, const T d[3], const T w[6], const T z[3]);

// What one queued hit adds: the 28 terms when linearizing, d^T W d when
// evaluating (z is then unused), the latter with the same operations as the
// first term of the former, so evaluate's e at a pose is linearize's e at that
// pose bit for bit (a Levenberg-Marquardt step compares the two)
template <int MODE, typename T, typename A>
__device__ __forceinline__ void add_hit(A& acc, const T d[3], const T w[6], const T z[3]) {
    if constexpr (MODE == kLin) {
        add_lin_terms(acc, d, w, z);
    } else {
        T u[3];
        sym3_mul(w, d, u);
        acc.add2(0, d[0], u[0], d[1], u[1]);
        acc.add(0, d[2] * u[2]);
    }
}

template <typename T, typename A>
__device__ __forceinline__ void add_lin_terms(A& acc, const T d[3], const T w[6], const T z[3]) {
    T u[3];
    sym3_mul(w, d, u);
    acc.add2(0, d[0], u[0], d[1], u[1]);
    acc.add(0, d[2] * u[2]);
    // P = (z)x W
    const T P00 = -z[2] * w[1] + z[1] * w[2], P01 = -z[2] * w[3] + z[1] * w[4], P02 = -z[2] * w[4] + z[1] * w[5];
    const T P10 = z[2] * w[0] - z[0] * w[2], P11 = z[2] * w[1] - z[0] * w[4], P12 = z[2] * w[2] - z[0] * w[5];
    const T P20 = -z[1] * w[0] + z[0] * w[1], P21 = -z[1] * w[1] + z[0] * w[3], P22 = -z[1] * w[2] + z[0] * w[4];
    // H''_ww = -P (z)x
    acc.add2(1 + tri(0, 0), -P01, z[2], P02, z[1]);
    acc.add2(1 + tri(0, 1), P00, z[2], -P02, z[0]);
    acc.add2(1 + tri(0, 2), -P00, z[1], P01, z[0]);
    acc.add2(1 + tri(1, 1), P10, z[2], -P12, z[0]);
    acc.add2(1 + tri(1, 2), -P10, z[1], P11, z[0]);
    acc.add2(1 + tri(2, 2), -P20, z[1], P21, z[0]);
    // H''_wv = P
    acc.add(1 + tri(0, 3), P00);
    acc.add(1 + tri(0, 4), P01);
    acc.add(1 + tri(0, 5), P02);
    acc.add(1 + tri(1, 3), P10);
    acc.add(1 + tri(1, 4), P11);
    acc.add(1 + tri(1, 5), P12);
    acc.add(1 + tri(2, 3), P20);
    acc.add(1 + tri(2, 4), P21);
    acc.add(1 + tri(2, 5), P22);
    // H''_vv = W
    acc.add(1 + tri(3, 3), w[0]);
    acc.add(1 + tri(3, 4), w[1]);
    acc.add(1 + tri(3, 5), w[2]);
    acc.add(1 + tri(4, 4), w[3]);
    acc.add(1 + tri(4, 5), w[4]);
    acc.add(1 + tri(5, 5), w[5]);
    // b'' = [u x z; -u]
    acc.add2(22, u[1], z[2], -u[2], z[1]);
    acc.add2(23, u[2], z[0], -u[0], z[2]);
    acc.add2(24, u[0], z[1], -u[1], z[0]);
    acc.add(25, -u[0]);
    acc.add(26, -u[1]);
    acc.add(27, -u[2]);
}

// The fields of one level that the probe reads for every chunk.
// Keys are formed biased by 8192 (the lookup's unsigned form): the coarse
// anchor key kb of a chunk becomes (kb + (8192 >> s)) << s at a level s
// halvings finer, and the key box's corner is biased the same way.
struct ProbeLevel {
    const uint64_t* slots;
    uint32_t log2cap, log2scale;
    uint32_t kbias;       // 8192 >> log2scale
    float inv_r, r;
    uint32_t kbox0u[3];   // key box corner + 8192
    uint32_t kboxw[3];
    const float* rec32;   // read by the hit terms of the first level
    double r64;
    __device__ __forceinline__ explicit ProbeLevel(const LevelDesc& lv)
        : slots(lv.slots), log2cap(lv.log2cap), log2scale((uint32_t)lv.log2scale),
          kbias((uint32_t)kKeyBias >> (uint32_t)lv.log2scale), inv_r(lv.inv_r), r(lv.r),
          kbox0u{(uint32_t)(lv.kbox0[0] + kKeyBias), (uint32_t)(lv.kbox0[1] + kKeyBias),
                 (uint32_t)(lv.kbox0[2] + kKeyBias)},
          kboxw{lv.kboxw[0], lv.kboxw[1], lv.kboxw[2]}, rec32(lv.rec32), r64(lv.r64) {}
};

// Per-tile chunk data in LDS.  At 4 waves per SIMD a CU holds at most 16
// waves, so even one-wave workgroups need at most 16 x 9 KB of the 160 KB.
// The FP32 data of one chunk, read together from one LDS address.
struct ChunkLds {
    float frac32[3];   // anchor position inside its coarse voxel, FP32 (voxel keys; in voxel units in one-level
                       // compacted kernels)
    int32_t kb[3];     // coarse relative key of the anchor (biased by 8192 in one-level kernels)
    float za[3];       // R (anchor - o_s)
    float vc[3];       // anchor - T^-1 c (surface validation)
};
struct TileShared {
    double frac[kMaxTileChunks * 3];   // anchor position inside its coarse voxel, FP64 (kC32; minus r/2 in
                                       // one-level compacted kernels)
    ChunkLds cd[kMaxTileChunks];
    int32_t live[kMaxTileChunks];      // the chunks the waves walk, in chunk order
    int32_t nlive;
    int32_t walked;                    // source points in those chunks
    uint8_t reach[kMaxTileChunks];     // kChunkCulled / kChunkStraddles / kChunkInside
};

// Per-wave queue of (point, level) hits of the compacted linearization and
// evaluation: the probe (keys, bounding box, block-table lookup) runs on every
// point, the expensive part (record gather, fused covariance and its inverse,
// residual, the 28 terms or e) only on full waves of hits.  Ring of 128 entries: a push adds at
// most 64 (one level of one chunk) and once 64 are queued a full wave is
// drained before the next push, so at most 127 are ever held.  The FP64 mode leaves x, y, z
// unused (its drain re-reads the FP64 position).
constexpr int kQueue = 128;
static_assert(kMaxTilePoints < 65536, "per-tile counts are packed in 16 bits");
struct HitQueue {
    float x[kQueue], y[kQueue], z[kQueue];   // point offset from its chunk anchor (compensated mode)
    int32_t pt[kQueue];                      // point index in the source (internal order)
    int32_t rec[kQueue];                     // voxel record index
    int32_t cl[kQueue];                      // chunk in tile (bits 2..) and level (bits 0..1)
};

// Raw per-point inputs of one precision mode, loaded one chunk ahead.
template <int PREC>
struct RawPoint {
    float x[3];   // kC32: offset from the chunk anchor; kN32: absolute position
};
template <>
struct RawPoint<kF64> {
    double x[3];
};

// Point `base + lane` of a source (internal order); base is the chunk's first
// point (uniform), so the addresses are a scalar base plus the lane's offset.
// Pad points (up to n_pad) are stored as zeros, so every lane may load.
template <int PREC>
__device__ __forceinline__ void load_point(const FactorDesc* __restrict__ Fp, __amdgpu_buffer_rsrc_t xr,
                                           uint32_t base, int64_t n_pad, uint32_t lane, RawPoint<PREC>& p) {
    if constexpr (PREC == kC32) {
        // buffer loads: the component's and chunk's offset is a scalar, the lane's a constant
#pragma unroll
        for (int a = 0; a < 3; ++a) p.x[a] = rsrc_load_f32(xr, lane * 4u, (uint32_t)(a * n_pad + base) * 4u);
    } else if constexpr (PREC == kN32) {
#pragma unroll
        for (int a = 0; a < 3; ++a) p.x[a] = load_off<float>(Fp->axyz + a * n_pad + base, lane * 4u);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) p.x[a] = load_off<double>(Fp->xyz64 + a * n_pad + base, lane * 8u);
    }
}

// S = R C R^T of point i.  The covariance is read only here, at the point's first
// hit: most points find no voxel, and their covariances are never loaded.
template <int PREC, typename TS, typename T>
__device__ __forceinline__ void point_S(const FactorDesc* __restrict__ Fp, int64_t i, int64_t n_pad,
                                        const double* P, const T* R, TS* S) {
    if constexpr (PREC == kC32) {
        // the covariances as a buffer (6 x n_pad floats): one lane offset, scalar component offsets
        const __amdgpu_buffer_rsrc_t cr = raw_rsrc(Fp->cov, (uint32_t)(6 * n_pad * (int64_t)sizeof(float)));
        double R64[9], C64[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) C64[k] = (double)rsrc_load_f32(cr, (uint32_t)i * 4u, (uint32_t)(k * n_pad) * 4u);
#pragma unroll
        for (int k = 0; k < 9; ++k) R64[k] = P[k];
        rotate_cov(R64, C64, S);
    } else if constexpr (PREC == kN32) {
        const auto Cv = gbl(Fp->cov);
        float C[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) C[k] = Cv[k * n_pad + i];
        rotate_cov(R, C, S);
    } else {
        const auto Cv = gbl(Fp->cov64);
        double C[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) C[k] = Cv[k * n_pad + i];
        rotate_cov(R, C, S);
    }
}

// Gradient of point i (internal order) of a factor: a source used by this
// factor only is written in place (caller order); a source shared with other
// factors gets this factor's own rows in the per-factor buffer, summed per
// source in factor order by k_grad_combine, so the result does not depend on
// which workgroup finished first.
__device__ __forceinline__ void write_point_grad(const FactorDesc* __restrict__ Fp, int64_t i, void* grad_points,
                                                 void* grad_slab, int32_t dtype, double g0, double g1, double g2) {
    const bool own = Fp->grad_slab < 0;
    const int64_t row = (own ? Fp->grad_offset : Fp->grad_slab) + Fp->perm[i];
    void* base = own ? grad_points : grad_slab;
    if (dtype == 0) {
        float* g = (float*)base + 3 * row;
        g[0] = (float)g0;
        g[1] = (float)g1;
        g[2] = (float)g2;
    } else {
        double* g = (double*)base + 3 * row;
        g[0] = g0;
        g[1] = g1;
        g[2] = g2;
    }
}

// Where the backward pass writes point gradients: the upstream gradient of the
// factor's e, the caller's rows, the per-factor rows of shared sources and the
// element type (0 FP32, 1 FP64).  Unused when linearizing or evaluating.
struct GradOut {
    double ge;
    void* points;
    void* slab;
    int32_t dtype;
};

// Terms of one queued hit (compensated mode): the same arithmetic as the
// uncompacted path, with the point's chunk and level taken from the entry.
// SC (one-level kernels): R is the rotation scaled by 1/r, the chunk data hold
// the anchor remainder scaled by 1/r (FP32, for the key) and minus r/2 (FP64,
// for the residual), and the entry holds the chunk's byte offset in the LDS
// chunk array.  The fused covariance is formed with the voxel's covariance
// added inside the rotation's last multiply-adds, and the residual as one FMA
// chain starting from the voxel centre.
template <int MODE, bool SC, typename A>
__device__ __forceinline__ void cmp_hit_terms(A& acc, const FactorDesc* __restrict__ Fp, const TileShared& sh,
                                              const ProbeLevel& pl0, const double* P, const float* R, int64_t n_pad,
                                              float dx, float dy, float dz, int32_t i, int32_t v, int32_t cl,
                                              const GradOut& go) {
    if constexpr (SC) {
        static_assert(sizeof(ChunkLds) == 48, "the FP64 remainders of a chunk sit at half its byte offset");
        const ChunkLds& cd = *reinterpret_cast<const ChunkLds*>(reinterpret_cast<const char*>(sh.cd) + cl);
        const double* fh = reinterpret_cast<const double*>(reinterpret_cast<const char*>(sh.frac) + (cl >> 1));
        // the point's covariance (read only here: most points find no voxel) and
        // the voxel record: all ten loads are issued before any result is used
        const __amdgpu_buffer_rsrc_t cr = raw_rsrc(Fp->cov, (uint32_t)(6 * n_pad * (int64_t)sizeof(float)));
        float C32[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) C32[k] = rsrc_load_f32(cr, (uint32_t)i * 4u, (uint32_t)(k * n_pad) * 4u);
        const uint32_t ro = (uint32_t)v * (uint32_t)(kRec32 * sizeof(float));
        const f32x3 q0 = load_off<f32x3>(pl0.rec32, ro);   // mean - centre (the count is not needed)
        const f64x2 cva = load_off<f64x2>(pl0.rec32, ro + 16u), cvb = load_off<f64x2>(pl0.rec32, ro + 32u),
                    cvc = load_off<f64x2>(pl0.rec32, ro + 48u);
        // the chunk's data (LDS), read while the loads are in flight
        float f32[3], za[3];
        double fhv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            f32[a] = cd.frac32[a];
            za[a] = cd.za[a];
            fhv[a] = fh[a];
        }
        __builtin_amdgcn_sched_barrier(0);
        double C64[6], R64[9];
#pragma unroll
        for (int k = 0; k < 6; ++k) C64[k] = (double)C32[k];
#pragma unroll
        for (int k = 0; k < 9; ++k) R64[k] = P[k];
        int32_t jk[3];
        float z[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float yl = chunk_pos32(f32[a], R[3 * a], R[3 * a + 1], R[3 * a + 2], dx, dy, dz);
            jk[a] = floor_i32(yl);
            z[a] = fmaf(yl - f32[a], pl0.r, za[a]);
        }
        const double Ct[6] = {cva.x, cva.y, cvb.x, cvb.y, cvc.x, cvc.y};
        double M[6], S[6];
        if constexpr (MODE == kBwd) {
            // the backward terms need R C R^T itself
            rotate_cov(R64, C64, S);
#pragma unroll
            for (int k = 0; k < 6; ++k) M[k] = Ct[k] + S[k];
        } else {
            rotate_cov_add(R64, C64, Ct, M);
        }
        float W[6];
        sym3_inverse_f32(M, W);
        // d = mu~ - y in FP64: (voxel mean - centre) - ((anchor remainder - r/2) - jk r + R offset)
        const double ddx = dx, ddy = dy, ddz = dz;
        const float mv[3] = {q0.x, q0.y, q0.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double base = fma(-(double)jk[a], pl0.r64, fhv[a]) - (double)mv[a];
            d[a] = -(float)fma(P[3 * a + 2], ddz, fma(P[3 * a + 1], ddy, fma(P[3 * a], ddx, base)));
        }
        if constexpr (MODE == kBwd) {
            // de/dxi terms (target orientation) and the point's row -2 R^T u (source
            // frame; R from the FP64 pose, as the terms' rotation here is scaled by 1/r)
            float u[3], Sf[6], Su[3];
            sym3_mul(W, d, u);
#pragma unroll
            for (int k = 0; k < 6; ++k) Sf[k] = (float)S[k];
            sym3_mul(Sf, u, Su);
            const float q0 = z[0] + Su[0], q1 = z[1] + Su[1], q2 = z[2] + Su[2];
            acc.add(0, 2.0f * (u[1] * q2 - u[2] * q1));
            acc.add(1, 2.0f * (u[2] * q0 - u[0] * q2));
            acc.add(2, 2.0f * (u[0] * q1 - u[1] * q0));
            acc.add(3, -2.0f * u[0]);
            acc.add(4, -2.0f * u[1]);
            acc.add(5, -2.0f * u[2]);
            if (go.points != nullptr) {
                const double u0 = u[0], u1 = u[1], u2 = u[2];
                write_point_grad(Fp, i, go.points, go.slab, go.dtype, go.ge * (-2.0 * (P[0] * u0 + P[3] * u1 + P[6] * u2)),
                                 go.ge * (-2.0 * (P[1] * u0 + P[4] * u1 + P[7] * u2)),
                                 go.ge * (-2.0 * (P[2] * u0 + P[5] * u1 + P[8] * u2)));
            }
        } else {
            add_hit<MODE>(acc, d, W, z);
        }
        return;
    }
    const int c = cl >> 2, l = cl & 3;
    // the level's record array, 1/r and r: the first level's come from scalar
    // registers, so its record gather does not wait on a descriptor load
    const float* rec_base = pl0.rec32;
    float inv_r = pl0.inv_r;
    double r64 = pl0.r64;
    if (l != 0) {
        const LevelDesc& lv = Fp->lv[l];
        rec_base = lv.rec32;
        inv_r = lv.inv_r;
        r64 = lv.r64;
    }
    const uint32_t ro = (uint32_t)v * (uint32_t)(kRec32 * sizeof(float));
    const f32x4 q0 = load_off<f32x4>(rec_base, ro);
    const f64x2 cva = load_off<f64x2>(rec_base, ro + 16u), cvb = load_off<f64x2>(rec_base, ro + 32u),
                cvc = load_off<f64x2>(rec_base, ro + 48u);
    double S[6];
    point_S<kC32>(Fp, (int64_t)i, n_pad, P, R, S);
    int32_t jk[3];
    float z[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float yl = chunk_pos32(sh.cd[c].frac32[a], R[3 * a], R[3 * a + 1], R[3 * a + 2], dx, dy, dz);
        jk[a] = floor_i32(yl * inv_r);
        z[a] = sh.cd[c].za[a] + fmaf(R[3 * a + 2], dz, fmaf(R[3 * a + 1], dy, R[3 * a] * dx));
    }
    double M[6], W64[6];
    M[0] = cva.x + S[0];
    M[1] = cva.y + S[1];
    M[2] = cvb.x + S[2];
    M[3] = cvb.y + S[3];
    M[4] = cvc.x + S[4];
    M[5] = cvc.y + S[5];
    sym3_inverse(M, W64);
    float W[6], d[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) W[k] = (float)W64[k];
    const float mv[3] = {q0.x, q0.y, q0.z};
    // y - voxel centre in FP64: (anchor remainder - r/2) + R offset - jk r (jk r exact)
    const double ddx = dx, ddy = dy, ddz = dz;
    const double half = 0.5 * r64;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double t = fma(P[3 * a + 2], ddz, fma(P[3 * a + 1], ddy, fma(P[3 * a], ddx, sh.frac[3 * c + a] - half)));
        d[a] = (float)((double)mv[a] - fma(-(double)jk[a], r64, t));
    }
    add_hit<MODE>(acc, d, W, z);
}

// Terms of one queued hit in the FP64 mode: the point is re-read from the
// FP64 positions (it was read one drain ago, so the load hits the caches) and
// the arithmetic is the uncompacted FP64 path's.
template <int MODE, typename A>
__device__ __forceinline__ void cmp_hit_terms64(A& acc, const FactorDesc* __restrict__ Fp, const double* P,
                                                const double* R, const double* tt, int64_t n_pad, int32_t i,
                                                int32_t v, int32_t cl) {
    const LevelDesc& lv = Fp->lv[cl & 3];
    const auto X = gbl(Fp->xyz64);
    const double x[3] = {X[i], X[n_pad + i], X[2 * n_pad + i]};
    const auto r2 = gbl(reinterpret_cast<const f64x2*>(lv.rec64 + (int64_t)v * kRec64));
    const f64x2 q0 = r2[0], q1 = r2[1], q2 = r2[2], q3 = r2[3], q4 = r2[4];
    double S[6];
    point_S<kF64>(Fp, (int64_t)i, n_pad, P, R, S);
    double z[3], d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) z[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2];
    d[0] = q0.x - (z[0] + tt[0]);
    d[1] = q0.y - (z[1] + tt[1]);
    d[2] = q1.x - (z[2] + tt[2]);
    const double M[6] = {q1.y + S[0], q2.x + S[1], q2.y + S[2], q3.x + S[3], q3.y + S[4], q4.x + S[5]};
    double W[6];
    sym3_inverse(M, W);
    add_hit<MODE>(acc, d, W, z);
}

// One queued hit, by precision mode.
template <int MODE, int PREC, bool SC, typename A, typename T>
__device__ __forceinline__ void drain_hit(A& acc, const FactorDesc* __restrict__ Fp, const TileShared& sh,
                                          const ProbeLevel& pl0, const double* P, const T* R, const T* tt,
                                          int64_t n_pad, const HitQueue& Q, int e, const GradOut& go) {
    if constexpr (PREC == kC32)
        cmp_hit_terms<MODE, SC>(acc, Fp, sh, pl0, P, R, n_pad, Q.x[e], Q.y[e], Q.z[e], Q.pt[e], Q.rec[e], Q.cl[e], go);
    else
        cmp_hit_terms64<MODE>(acc, Fp, P, R, tt, n_pad, Q.pt[e], Q.rec[e], Q.cl[e]);
}

// Register budget: 4 waves per SIMD (<= 128 VGPRs) for the FP32 modes; the
// FP64 mode needs more and runs at what its register count allows.
template <int PREC, bool KH>
constexpr int waves_per_eu() { return (PREC == kF64 || KH) ? 1 : 4; }
// the FP32 kernels are held at exactly four (the scheduler then keeps loads in
// flight instead of saving registers for a fifth); the others may run up to the
// eight a SIMD holds, so their scheduler still works for occupancy
template <int PREC, bool KH>
constexpr int waves_per_eu_max() { return waves_per_eu<PREC, KH>() == 4 ? 4 : 8; }

// Every point of chunk cg lies in a ball around the anchor and in a box of
// the source frame, both stored with the chunk.  In the target frame (anchor
// at ya) the ball keeps its radius and the box is covered by the axis-aligned
// box of half extents |R| h.  A chunk whose ball or box misses the key box of
// every level has no correspondence (culled); a chunk whose ball lies inside
// the key box of every level has no point outside them, so its points skip the
// per-point box test.  The margins (1e-3 m + 1e-5 relative) cover FP32 key
// positions and the FP32 rounding of the stored offsets.
constexpr int kChunkCulled = 0, kChunkStraddles = 1, kChunkInside = 2;
constexpr int kInsideFlag = 1 << 16;   // in a live-list entry: the chunk is inside every key box
__device__ __forceinline__ int chunk_state(const FactorDesc* __restrict__ Fp, const double* P, const double ya[3],
                                           int64_t cg, int L) {
    const auto cb = gbl(Fp->cbound + 8 * cg);
    const double rr = (double)cb[3] * (1.0 + 1e-5) + 1e-3;
    double yc[3], ex[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        yc[i] = ya[i] + (P[3 * i] * cb[0] + P[3 * i + 1] * cb[1] + P[3 * i + 2] * cb[2]);
        ex[i] = (fabs(P[3 * i]) * cb[4] + fabs(P[3 * i + 1]) * cb[5] + fabs(P[3 * i + 2]) * cb[6]) * (1.0 + 1e-5) +
                1e-3;
    }
    bool reach = false, inside = true;
    for (int l = 0; l < L; ++l) {
        const LevelDesc& lv = Fp->lv[l];
        double d2 = 0.0;
        bool box = true;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double g = fmax(0.0, fmax(lv.blo[i] - ya[i], ya[i] - lv.bhi[i]));
            d2 += g * g;
            box = box && (yc[i] + ex[i] >= lv.blo[i]) && (yc[i] - ex[i] <= lv.bhi[i]);
            inside = inside && (ya[i] - rr >= lv.blo[i]) && (ya[i] + rr <= lv.bhi[i]);
        }
        reach |= (d2 <= rr * rr) && box;
    }
    return !reach ? kChunkCulled : (inside ? kChunkInside : kChunkStraddles);
}

// Point-gradient rows of the shared sources: row k of source s is the sum over
// its factors, in factor order, of their rows k in the per-factor buffer
// (FP64 sums of the per-factor values).  One thread per row.
__global__ void k_grad_combine(const SharedSrc* __restrict__ ss, int32_t S, int64_t rows,
                               const int64_t* __restrict__ slab_off, const void* __restrict__ slab,
                               void* __restrict__ out, int32_t dtype) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    int lo = 0, hi = S - 1;   // last shared source whose rows start at or before r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ss[mid].row0 <= r) lo = mid;
        else hi = mid - 1;
    }
    const SharedSrc q = ss[lo];
    const int64_t k = r - q.row0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int32_t j = q.f0; j < q.f1; ++j) {
        const int64_t o = 3 * (slab_off[j] + k);
        if (dtype == 0) {
            const float* g = (const float*)slab + o;
            a0 += (double)g[0];
            a1 += (double)g[1];
            a2 += (double)g[2];
        } else {
            const double* g = (const double*)slab + o;
            a0 += g[0];
            a1 += g[1];
            a2 += g[2];
        }
    }
    const int64_t w = 3 * (q.grad_offset + k);
    if (dtype == 0) {
        float* g = (float*)out + w;
        g[0] = (float)a0;
        g[1] = (float)a1;
        g[2] = (float)a2;
    } else {
        double* g = (double*)out + w;
        g[0] = a0;
        g[1] = a1;
        g[2] = a2;
    }
}

// Pose staging: FP32 copies of every factor's R and t (16 floats per factor),
// read by the tile kernel through uniform (scalar) loads.
__global__ void k_stage_poses(int64_t F, const double* __restrict__ poses, float* __restrict__ posef) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F * 16) return;
    const int64_t f = i / 16, k = i % 16;
    posef[i] = (k < 12) ? (float)poses[12 * f + k] : 0.0f;
}

// VAL: surface validation (a compile-time switch, so that batches without it
// carry none of its state through the point loop).  LM: the most levels the
// point loop is compiled for (1 for single-level batches, whose kernel then
// holds no state of the other levels; else kMaxLevels).
template <int MODE, int PREC, int BLOCK, bool KH, bool VAL, int LM>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(waves_per_eu<PREC, KH>(), waves_per_eu_max<PREC, KH>()))) void k_tiles(
    const FactorDesc* __restrict__ fac, const Tile* __restrict__ tiles, int32_t t_begin, int32_t t_end,
    const double* __restrict__ poses, const float* __restrict__ posef, double* __restrict__ partials,
    uint32_t* __restrict__ counter, const double* __restrict__ grad_e,
    void* __restrict__ grad_points, void* __restrict__ grad_slab, int32_t points_dtype, int32_t interleave) {
    using T = typename PT<PREC>::T;
    constexpr bool validate = VAL;
    constexpr int NW = BLOCK / 64;
    constexpr bool KAHAN = KH && (PREC == kC32);
    constexpr int NT = (MODE == kLin) ? kTerms : (MODE == kBwd ? 6 : 1);
    // compacted hits: linearize in the compensated and FP64 modes, evaluate in
    // the compensated mode (the FP64 evaluate measured faster per lane), and the
    // one-level compensated backward pass (its caller zeroes the point-gradient
    // rows, so only points with a voxel write theirs)
    constexpr bool CMP = (MODE == kLin && (PREC == kC32 || PREC == kF64)) || (MODE == kEval && PREC == kC32) ||
                         (MODE == kBwd && PREC == kC32 && LM == 1 && !VAL && !KH);
    // chunks that cannot reach any level's key box are skipped (not in the
    // per-lane backward pass, which writes a gradient row for every point, nor
    // in the naive FP32 mode, whose absolute-coordinate keys can be off by more
    // than the culling margin far from the origin)
    constexpr bool SKIP = ((PREC == kC32 || PREC == kF64) && (MODE != kBwd || CMP));
    // a one-level kernel keeps the chunks' anchor keys biased by 8192 in LDS
    // (its only level is the coarse one, so they are the lookup's keys as they are)
    constexpr int32_t KBB = (LM == 1) ? kKeyBias : 0;
    // one-level compacted kernels: positions in voxel units (the rotation and
    // the anchor remainders scaled by 1/r), so keys need no multiply
    constexpr bool SC = CMP && PREC == kC32 && LM == 1;
    // the compacted probes issue a chunk's table loads and drain a full wave of
    // earlier hits while they are in flight, then push the chunk's hits; the
    // compensated kernel with validation (short of registers for it) drains
    // after the push instead.  Either way a drain takes the queue's oldest 64
    // entries, so both orders process the same hits in the same lanes.
    constexpr bool DRAIN_EARLY = !(PREC == kC32 && VAL);
    __shared__ TileShared sh;
    using QueueT = typename std::conditional<CMP, HitQueue, int32_t>::type;
    __shared__ QueueT s_q[CMP ? NW : 1];
    __shared__ double s_red[NW][kRow];
    __shared__ int32_t s_tile;
    const int lane = threadIdx.x & 63;
    // wave index as a uniform (scalar) value, so chunk indices and per-chunk LDS
    // addresses are computed once per wave, not per lane
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware work distribution: the tiles are split into kParts partitions with
    // one counter each; workgroups are dispatched round-robin over the XCDs, so
    // workgroup b starts on partition b % kParts, i.e. on its XCD's partition.
    // Contiguous partitions give each XCD's L2 a narrow window of factors (which
    // share sources and targets); interleaved partitions (tile i in partition
    // i % kParts) keep all XCDs in one window, so the last-level cache holds a
    // single working set.  A workgroup whose partition is exhausted moves on to
    // the next one.
    const int32_t ntiles = t_end - t_begin;
    const int32_t span = (ntiles + kParts - 1) / kParts;
    int part = (int)(blockIdx.x % kParts);
    int tried = 0;

    for (;;) {
        if (threadIdx.x == 0) {
            int32_t take = -1;
            while (tried < kParts) {
                if (interleave) {
                    const int32_t cnt = ntiles > part ? (ntiles - part + kParts - 1) / kParts : 0;
                    if (cnt > 0) {
                        const uint32_t k = atomicAdd(counter + part, 1u);
                        if (k < (uint32_t)cnt) {
                            take = t_begin + part + kParts * (int32_t)k;
                            break;
                        }
                    }
                } else {
                    const int32_t lo = t_begin + part * span;
                    const int32_t hi = min(lo + span, t_end);
                    if (lo < hi) {
                        const uint32_t k = atomicAdd(counter + part, 1u);
                        if (k < (uint32_t)(hi - lo)) {
                            take = lo + (int32_t)k;
                            break;
                        }
                    }
                }
                part = (part + 1) % kParts;
                ++tried;
            }
            s_tile = take;
        }
        __syncthreads();
        const int32_t t = __builtin_amdgcn_readfirstlane(s_tile);
        if (t < 0) break;
        const Tile tile = tiles[t];
        const FactorDesc* __restrict__ Fp = fac + tile.factor;
        const int64_t n = Fp->n, n_pad = Fp->n_pad;
        const int L = Fp->L;
        const double* P = poses + 12 * tile.factor;
        // pose (uniform): FP32 copies from the staged block, FP64 straight from the poses
        T R[9], tt[3];
        if constexpr (PREC == kF64) {
#pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = P[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) tt[k] = P[9 + k];
        } else if constexpr (SC) {
            // R / r (the map's one level), uniform
            const double ir = Fp->lv[0].inv_r64;
#pragma unroll
            for (int k = 0; k < 9; ++k)
                R[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)(P[k] * ir))));
#pragma unroll
            for (int k = 0; k < 3; ++k) tt[k] = 0.0f;
        } else {
            const float* Pf = posef + 16 * (int64_t)tile.factor;
#pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = Pf[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) tt[k] = Pf[9 + k];
        }
        // T^-1 c (source frame) for validation, in FP64
        double cs[3] = {0, 0, 0};
        if (validate) {
            const double dc0 = Fp->viewpoint[0] - P[9], dc1 = Fp->viewpoint[1] - P[10], dc2 = Fp->viewpoint[2] - P[11];
#pragma unroll
            for (int i = 0; i < 3; ++i) cs[i] = P[i] * dc0 + P[3 + i] * dc1 + P[6 + i] * dc2;
        }
        // ---------------------------------------------------------------- per-tile state
        Acc<T, KAHAN, NT> acc;
        acc.zero();
        // points with a voxel and table lookups per level: per lane, or in the
        // compacted paths wave-uniform totals packed two levels per word (level l
        // in bits 16 (l % 2) of word l / 2; a tile has fewer than 65536 points);
        // source points and chunks walked (uniform)
        int32_t inl[kMaxLevels] = {0, 0, 0, 0};
        int32_t prb[kMaxLevels] = {0, 0, 0, 0};
        uint32_t inl2[2] = {0u, 0u}, prb2[2] = {0u, 0u};
        int32_t walked_pts = 0, walked_chunks = 0;
        double ge = 0.0;
        if constexpr (MODE == kBwd) ge = grad_e[tile.factor];
        const GradOut go{ge, grad_points, grad_slab, points_dtype};

        // this wave's hit queue (wave-uniform); the head is 0 or 64 (full waves are
        // drained, and the queue restarts at 0 once a batch's rest is drained), so a
        // drained wave of entries is head + lane with no wrap
        int q_head = 0, q_count = 0;

        // the first level's probe constants, loaded once per tile (uniform)
        const ProbeLevel pl0(Fp->lv[0]);
        // one full wave of queued hits, the oldest 64 (head + lane, no wrap)
        auto drain_full = [&](const QueueT& Q) {
            if constexpr (CMP) {
                if (q_count >= kChunk) {
                    __builtin_amdgcn_wave_barrier();
                    drain_hit<MODE, PREC, SC>(acc, Fp, sh, pl0, P, R, tt, n_pad, Q, q_head + lane, go);
                    q_head = (q_head + kChunk) & (kQueue - 1);
                    q_count -= kChunk;
                    __builtin_amdgcn_wave_barrier();
                }
            }
        };
        // the source's positions as a buffer (3 x n_pad floats; sources hold fewer than 2^27 points)
        const __amdgpu_buffer_rsrc_t xr = raw_rsrc(Fp->dxyz, (uint32_t)(3 * n_pad * (int64_t)sizeof(float)));
        const int32_t n32 = (int32_t)n;
        // The tile's chunks are taken in batches of up to kMaxTileChunks (the
        // per-chunk data held in LDS); the lane sums run on across batches, so a
        // tile of several batches is reduced once.
        for (int sb0 = 0; sb0 < tile.nchunks; sb0 += kMaxTileChunks) {
            const int nch = min(kMaxTileChunks, tile.nchunks - sb0);
            const int chunk0 = tile.chunk0 + sb0;
            // ---------------------------------------------------------------- prologue: chunk anchors (kC32)
            if constexpr (PREC == kC32) {
                const LevelDesc& top = Fp->lv[L - 1];
                for (int c = threadIdx.x; c < nch; c += BLOCK) {
                    const auto a = gbl(Fp->anchor + 3 * (int64_t)(chunk0 + c));
                    const double a0 = a[0], a1 = a[1], a2 = a[2];
                    const double o0 = a0 - Fp->src_origin[0], o1 = a1 - Fp->src_origin[1], o2 = a2 - Fp->src_origin[2];
                    const double av[3] = {a0, a1, a2};
                    double ya[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        double fr;
                        int32_t kb;
                        ya[i] = anchor_split(P, av, i, top.r64, top.inv_r64, top.K0[i], &fr, &kb);
                        if constexpr (SC) {
                            sh.frac[3 * c + i] = fr - 0.5 * top.r64;
                            sh.cd[c].frac32[i] = (float)(fr * top.inv_r64);
                        } else {
                            sh.frac[3 * c + i] = fr;
                            sh.cd[c].frac32[i] = (float)fr;
                        }
                        sh.cd[c].kb[i] = kb + KBB;
                        sh.cd[c].za[i] = (float)(P[3 * i] * o0 + P[3 * i + 1] * o1 + P[3 * i + 2] * o2);
                    }
                    if (validate) {
                        sh.cd[c].vc[0] = (float)(a0 - cs[0]);
                        sh.cd[c].vc[1] = (float)(a1 - cs[1]);
                        sh.cd[c].vc[2] = (float)(a2 - cs[2]);
                    }
                    if constexpr (SKIP) sh.reach[c] = (uint8_t)chunk_state(Fp, P, ya, chunk0 + c, L);
                }
                __syncthreads();
            } else if constexpr (SKIP) {
                for (int c = threadIdx.x; c < nch; c += BLOCK) {
                    const auto a = gbl(Fp->anchor + 3 * (int64_t)(chunk0 + c));
                    double ya[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) ya[i] = fma(P[3 * i + 2], a[2], fma(P[3 * i + 1], a[1], P[3 * i] * a[0])) + P[9 + i];
                    sh.reach[c] = (uint8_t)chunk_state(Fp, P, ya, chunk0 + c, L);
                }
                __syncthreads();
            }
            // the list of chunks to walk (kept in chunk order)
            if (wave == 0) {
                int cnt = 0;
                int32_t pts = 0;   // per lane: points of the chunks this lane kept
                for (int base = 0; base < nch; base += 64) {
                    const int c = base + lane;
                    bool keep = c < nch;
                    int flag = 0;
                    if constexpr (SKIP) {
                        const int st = keep ? (int)sh.reach[c] : kChunkCulled;
                        keep = st != kChunkCulled;
                        flag = st == kChunkInside ? kInsideFlag : 0;
                    }
                    const uint64_t m = __ballot(keep);
                    if (keep) {
                        sh.live[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = c | flag;
                        pts += (int32_t)min<int64_t>(kChunk, n - (int64_t)(chunk0 + c) * kChunk);
                    }
                    cnt += __popcll(m);
                }
                pts = wave_sum(pts);
                if (lane == 0) {
                    sh.nlive = cnt;
                    sh.walked = pts;
                }
            }
            __syncthreads();
            const int nlive = __builtin_amdgcn_readfirstlane(sh.nlive);
            // this wave walks entries wave, wave + NW, ... of the list; with two or
            // more waves they are at most 64, held one per lane and read by index
            int32_t mylive = 0;
            if constexpr (NW >= 2) {
                const int jj = wave + NW * lane;
                mylive = jj < nlive ? sh.live[jj] : 0;
            }
            auto live_chunk = [&](int j, int k) -> int {
                if constexpr (NW >= 2) return __builtin_amdgcn_readlane(mylive, k);
                else return __builtin_amdgcn_readfirstlane(sh.live[j]);
            };
            RawPoint<PREC> nxt;
            int cnext = 0;
            if (wave < nlive) {
                cnext = live_chunk(wave, 0);
                load_point<PREC>(Fp, xr, (uint32_t)(chunk0 + (cnext & (kInsideFlag - 1))) * kChunk, n_pad,
                                 (uint32_t)lane, nxt);
            }
            for (int j = wave, k = 0; j < nlive; j += NW, ++k) {
                const int c = cnext & (kInsideFlag - 1);
                // every point of the chunk is inside every level's key box (uniform)
                const bool inside = (cnext & kInsideFlag) != 0;
                // point index (sources hold fewer than 2^31 points) and the chunk's
                // point count (uniform: only a source's last chunk is partial)
                const uint32_t base = (uint32_t)(chunk0 + c) * kChunk;
                const int32_t i = (int32_t)(base + (uint32_t)lane);
                const int32_t npts = min(kChunk, n32 - (int32_t)base);
                const bool live = lane < npts;
                const RawPoint<PREC> cur = nxt;
                if (j + NW < nlive) {
                    cnext = live_chunk(j + NW, k + 1);
                    load_point<PREC>(Fp, xr, (uint32_t)(chunk0 + (cnext & (kInsideFlag - 1))) * kChunk, n_pad,
                                     (uint32_t)lane, nxt);
                }
                if constexpr (CMP && PREC == kF64) {
                    // ---- FP64 mode: probe every point, queue its hits, drain full waves
                    HitQueue& Q = s_q[wave];
                    const double x0 = cur.x[0], x1 = cur.x[1], x2 = cur.x[2];
                    double yl[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) yl[a] = (R[3 * a] * x0 + R[3 * a + 1] * x1 + R[3 * a + 2] * x2) + tt[a];
                    bool vis = live;
                    if (live && validate) {
                        const auto Nv = gbl(Fp->nrm64);
                        const double sv = (x0 - cs[0]) * Nv[i] + (x1 - cs[1]) * Nv[n_pad + i] + (x2 - cs[2]) * Nv[2 * n_pad + i];
                        vis = !(sv > 0.0);
                    }
#pragma unroll
                    for (int l = 0; l < LM; ++l) {
                        if (l >= L) break;
                        const LevelDesc& lv = Fp->lv[l];
                        int32_t kq[3];
                        bool in = vis;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const int64_t k = (int64_t)floor(yl[a] * lv.inv_r64) - lv.K0[a];
                            in &= (k >= lv.kmin[a]) & (k <= lv.kmax[a]);
                            kq[a] = (int32_t)k;
                        }
                        int32_t v = -1;
                        prb2[l >> 1] += (uint32_t)__popcll(__ballot(in)) << (16 * (l & 1));
                        // a full wave of earlier hits is processed while the table loads
                        // are in flight (see the compensated path below)
                        BlockProbe bp;
                        if (in)
                            lookup_issue(lv.slots, lv.log2cap, (uint32_t)(kq[0] + kKeyBias), (uint32_t)(kq[1] + kKeyBias),
                                         (uint32_t)(kq[2] + kKeyBias), bp);
                        if constexpr (DRAIN_EARLY) drain_full(Q);
                        if (in) v = lookup_finish(lv.slots, lv.log2cap, bp);
                        const bool hit = v >= 0;
                        const uint64_t mask = __ballot(hit);
                        inl2[l >> 1] += (uint32_t)__popcll(mask) << (16 * (l & 1));
                        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                        if (hit) {
                            const int e = (q_head + q_count + below) & (kQueue - 1);
                            Q.pt[e] = (int32_t)i;
                            Q.rec[e] = v;
                            Q.cl[e] = (c << 2) | l;
                        }
                        q_count += __popcll(mask);
                        if constexpr (!DRAIN_EARLY) drain_full(Q);
                    }
                    continue;
                } else if constexpr (CMP) {
                    // ---- probe every point, queue its hits, drain full waves of hits
                    HitQueue& Q = s_q[wave];
                    // issue priority up while the chunk's keys are formed and its table
                    // loads issued (lowered once they are out)
                    if constexpr (SC) __builtin_amdgcn_s_setprio(1);
                    const float dx = cur.x[0], dy = cur.x[1], dz = cur.x[2];
                    float yl[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        yl[a] = chunk_pos32(sh.cd[c].frac32[a], R[3 * a], R[3 * a + 1], R[3 * a + 2], dx, dy, dz);
                    bool vis = live;
                    if (live && validate) {
                        const auto Nv = gbl(Fp->nrm);
                        const float sv = (sh.cd[c].vc[0] + dx) * Nv[i] + (sh.cd[c].vc[1] + dy) * Nv[n_pad + i] +
                                         (sh.cd[c].vc[2] + dz) * Nv[2 * n_pad + i];
                        vis = !(sv > 0.0f);
                    }
#pragma unroll
                    for (int l = 0; l < LM; ++l) {
                        if (l >= L) break;
                        const LevelDesc& lv = Fp->lv[l];
                        const ProbeLevel pl = l == 0 ? pl0 : ProbeLevel(lv);
                        int32_t v = -1;
                        // biased key (coarse anchor key times the level ratio, a shift; a
                        // one-level kernel's only level is the coarse one) and the
                        // bounding-box test as one unsigned compare per axis, no branches
                        uint32_t ku[3];
                        bool in = vis;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const uint32_t fl = (uint32_t)floor_i32(SC ? yl[a] : yl[a] * pl.inv_r);
                            if constexpr (LM == 1) ku[a] = (uint32_t)sh.cd[c].kb[a] + fl;
                            else ku[a] = (((uint32_t)sh.cd[c].kb[a] + pl.kbias) << pl.log2scale) + fl;
                        }
                        // table lookups: inside the key boxes every visible point looks up
                        // (without validation, every point of the chunk: a uniform count)
                        uint32_t nlook;
                        if (inside) {
                            nlook = validate ? (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in)) : (uint32_t)npts;
                        } else {
#pragma unroll
                            for (int a = 0; a < 3; ++a) in &= (ku[a] - pl.kbox0u[a]) <= pl.kboxw[a];
                            nlook = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in));
                        }
                        prb2[l >> 1] += nlook << (16 * (l & 1));
                        // the table loads are issued (and the priority lowered), then a
                        // full wave of earlier hits is processed while they are in flight
                        // (the queue is FIFO and a drain takes its oldest 64 entries, so
                        // every drain sees the same hits in the same lanes as draining
                        // after the push would)
                        BlockProbe bp;
                        if (in) lookup_issue(pl.slots, pl.log2cap, ku[0], ku[1], ku[2], bp);
                        if constexpr (SC) __builtin_amdgcn_s_setprio(0);
                        if constexpr (DRAIN_EARLY) drain_full(Q);
                        if (in) v = lookup_finish(pl.slots, pl.log2cap, bp);
                        const bool hit = v >= 0;
                        const uint64_t mask = __builtin_amdgcn_ballot_w64(hit);
                        inl2[l >> 1] += (uint32_t)__popcll(mask) << (16 * (l & 1));
                        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                        if (hit) {
                            const int e = (q_head + q_count + below) & (kQueue - 1);
                            Q.x[e] = dx;
                            Q.y[e] = dy;
                            Q.z[e] = dz;
                            Q.pt[e] = (int32_t)i;
                            Q.rec[e] = v;
                            Q.cl[e] = SC ? c * (int)sizeof(ChunkLds) : (c << 2) | l;
                        }
                        q_count += __popcll(mask);
                        if constexpr (!DRAIN_EARLY) drain_full(Q);
                    }
                    continue;
                }
                if (!live) continue;
                // ---- load the point, transform it
                // yl: transformed position (kC32: relative to the anchor's coarse voxel corner)
                T x[3], z[3];
                T yl[3];          // transformed position (kC32: FP32, relative to the anchor's coarse voxel)
                bool vis = true;
                if constexpr (PREC == kC32) {
                    // Keys come from the FP32 position (its ~5e-7 m error only matters
                    // for points that close to a voxel face, where either voxel is a
                    // valid answer).  The residual d = mu~ - y cancels metre-scale
                    // positions down to centimetres, so for hits the offset from the
                    // anchor is rotated and placed relative to the voxel centre in FP64.
                    const float dx = cur.x[0], dy = cur.x[1], dz = cur.x[2];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        yl[a] = chunk_pos32(sh.cd[c].frac32[a], R[3 * a], R[3 * a + 1], R[3 * a + 2], dx, dy, dz);
                        z[a] = sh.cd[c].za[a] + fmaf(R[3 * a + 2], dz, fmaf(R[3 * a + 1], dy, R[3 * a] * dx));
                    }
                    x[0] = dx;
                    x[1] = dy;
                    x[2] = dz;
                    if (validate) {
                        const auto Nv = gbl(Fp->nrm);
                        const float s = (sh.cd[c].vc[0] + dx) * Nv[i] + (sh.cd[c].vc[1] + dy) * Nv[n_pad + i] +
                                        (sh.cd[c].vc[2] + dz) * Nv[2 * n_pad + i];
                        vis = !(s > 0.0f);
                    }
                } else if constexpr (PREC == kN32) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) x[a] = cur.x[a];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        z[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2];
                        yl[a] = z[a] + tt[a];
                    }
                    if (validate) {
                        const auto Nv = gbl(Fp->nrm);
                        const float s = (x[0] - (float)cs[0]) * Nv[i] + (x[1] - (float)cs[1]) * Nv[n_pad + i] +
                                        (x[2] - (float)cs[2]) * Nv[2 * n_pad + i];
                        vis = !(s > 0.0f);
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) x[a] = cur.x[a];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        z[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2];
                        yl[a] = z[a] + tt[a];
                    }
                    if (validate) {
                        const double s = (x[0] - cs[0]) * Fp->nrm64[i] + (x[1] - cs[1]) * Fp->nrm64[n_pad + i] +
                                         (x[2] - cs[2]) * Fp->nrm64[2 * n_pad + i];
                        vis = !(s > 0.0);
                    }
                }
                if (!vis) {
                    if constexpr (MODE == kBwd) {
                        if (grad_points != nullptr) write_point_grad(Fp, i, grad_points, grad_slab, points_dtype, 0.0, 0.0, 0.0);
                    }
                    continue;
                }
                // ---- per level: key, probe, terms
                // S = R C R^T, once per point (FP64 in the compensated mode, where the
                // fused covariance and its inverse are formed in FP64: both covariances
                // are near-singular, so FP32 rounding of either one would move W by
                // ~1e-4 relative along the surface normal)
                using TS = typename std::conditional<PREC == kC32, double, T>::type;
                TS S[6];
                bool haveS = false;
                T gp[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int l = 0; l < LM; ++l) {
                    if (l >= L) break;
                    const LevelDesc& lv = Fp->lv[l];
                    // relative key; a key outside the level's key bounding box (which also
                    // covers keys outside the packable range) has no voxel and is not probed
                    int32_t kq[3];
                    bool in = true;
                    int32_t jk[3];
                    T pc[3];   // absolute position (kN32, kF64)
                    if constexpr (PREC == kC32) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            jk[a] = floor_i32(yl[a] * lv.inv_r);
                            kq[a] = (int32_t)((uint32_t)(sh.cd[c].kb[a] - KBB) << lv.log2scale) + jk[a];
                            in &= (uint32_t)(kq[a] - lv.kbox0[a]) <= lv.kboxw[a];
                        }
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            int64_t k;
                            if constexpr (PREC == kN32) k = (int64_t)floorf(yl[a] * lv.inv_r) - lv.K0[a];
                            else k = (int64_t)floor(yl[a] * lv.inv_r64) - lv.K0[a];
                            in &= (k >= lv.kmin[a]) & (k <= lv.kmax[a]);
                            kq[a] = (int32_t)k;
                            pc[a] = yl[a];
                        }
                    }
                    if (!in) continue;
                    prb[l] += 1;
                    const int32_t v = lookup(lv.slots, lv.log2cap, kq[0], kq[1], kq[2]);
                    if (v < 0) continue;
                    inl[l] += 1;
                    if constexpr (MODE == kCount) continue;
                    T mv[3];
                    T W[6];
                    if constexpr (PREC == kC32) {
                        // the voxel record's loads are issued before the covariance's (first
                        // hit only), so the two round trips overlap
                        const float* rec = lv.rec32 + (int64_t)v * kRec32;
                        const f32x4 q0 = *gbl(reinterpret_cast<const f32x4*>(rec));
                        const auto c2 = gbl(reinterpret_cast<const f64x2*>(rec + 4));
                        const f64x2 cva = c2[0], cvb = c2[1], cvc = c2[2];
                        if (!haveS) {
                            point_S<PREC>(Fp, i, n_pad, P, R, S);
                            haveS = true;
                        }
                        mv[0] = q0.x; mv[1] = q0.y; mv[2] = q0.z;
                        double M[6], W64[6];
                        M[0] = cva.x + S[0];
                        M[1] = cva.y + S[1];
                        M[2] = cvb.x + S[2];
                        M[3] = cvb.y + S[3];
                        M[4] = cvc.x + S[4];
                        M[5] = cvc.y + S[5];
                        sym3_inverse(M, W64);
#pragma unroll
                        for (int k = 0; k < 6; ++k) W[k] = (float)W64[k];
                    } else {
                        T cvv[6];
                        if constexpr (PREC == kN32) {
                            const auto r4 = gbl(reinterpret_cast<const f32x4*>(lv.recN + (int64_t)v * kRecN));
                            const f32x4 q0 = r4[0], q1 = r4[1], q2 = r4[2];
                            mv[0] = q0.x; mv[1] = q0.y; mv[2] = q0.z;
                            cvv[0] = q0.w; cvv[1] = q1.x; cvv[2] = q1.y; cvv[3] = q1.z; cvv[4] = q1.w; cvv[5] = q2.x;
                        } else {
                            const auto r2 = gbl(reinterpret_cast<const f64x2*>(lv.rec64 + (int64_t)v * kRec64));
                            const f64x2 q0 = r2[0], q1 = r2[1], q2 = r2[2], q3 = r2[3], q4 = r2[4];
                            mv[0] = q0.x; mv[1] = q0.y; mv[2] = q1.x;
                            cvv[0] = q1.y; cvv[1] = q2.x; cvv[2] = q2.y; cvv[3] = q3.x; cvv[4] = q3.y; cvv[5] = q4.x;
                        }
                        if (!haveS) {
                            point_S<PREC>(Fp, i, n_pad, P, R, S);
                            haveS = true;
                        }
                        T M[6];
#pragma unroll
                        for (int k = 0; k < 6; ++k) M[k] = cvv[k] + S[k];
                        sym3_inverse(M, W);
                    }
                    T d[3];
                    if constexpr (PREC == kC32) {
                        // y relative to the centre of the voxel found above (FP64), then d = mu~ - y
                        const double ddx = cur.x[0], ddy = cur.x[1], ddz = cur.x[2];
                        const double half = 0.5 * lv.r64;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const double t = fma(P[3 * a + 2], ddz,
                                                 fma(P[3 * a + 1], ddy, fma(P[3 * a], ddx, sh.frac[3 * c + a] - half)));
                            d[a] = (float)((double)mv[a] - fma(-(double)jk[a], lv.r64, t));
                        }
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a) d[a] = mv[a] - pc[a];
                    }
                    if constexpr (MODE == kLin) {
                        add_lin_terms(acc, d, W, z);
                    } else if constexpr (MODE == kEval) {
                        T u[3];
                        sym3_mul(W, d, u);
                        acc.add(0, d[0] * u[0] + d[1] * u[1] + d[2] * u[2]);
                    } else {
                        T u[3], Su[3], Sf[6];
                        sym3_mul(W, d, u);
#pragma unroll
                        for (int k = 0; k < 6; ++k) Sf[k] = (T)S[k];
                        sym3_mul(Sf, u, Su);
                        const T q0 = z[0] + Su[0], q1 = z[1] + Su[1], q2 = z[2] + Su[2];
                        acc.add(0, T(2) * (u[1] * q2 - u[2] * q1));
                        acc.add(1, T(2) * (u[2] * q0 - u[0] * q2));
                        acc.add(2, T(2) * (u[0] * q1 - u[1] * q0));
                        acc.add(3, T(-2) * u[0]);
                        acc.add(4, T(-2) * u[1]);
                        acc.add(5, T(-2) * u[2]);
                        // de/dmu = -2 R^T u (source frame)
                        gp[0] += T(-2) * (R[0] * u[0] + R[3] * u[1] + R[6] * u[2]);
                        gp[1] += T(-2) * (R[1] * u[0] + R[4] * u[1] + R[7] * u[2]);
                        gp[2] += T(-2) * (R[2] * u[0] + R[5] * u[1] + R[8] * u[2]);
                    }
                }
                if constexpr (MODE == kBwd) {
                    if (grad_points != nullptr)
                        write_point_grad(Fp, i, grad_points, grad_slab, points_dtype, ge * (double)gp[0],
                                         ge * (double)gp[1], ge * (double)gp[2]);
                }
            }
            if constexpr (CMP) {
                // the queued hits refer to this batch's chunks: a full wave left by a
                // probe that drains before pushing, then the partial rest
                drain_full(s_q[wave]);
                if (q_count > 0) {
                    __builtin_amdgcn_wave_barrier();
                    if (lane < q_count) {
                        drain_hit<MODE, PREC, SC>(acc, Fp, sh, pl0, P, R, tt, n_pad, s_q[wave], (q_head + lane) & (kQueue - 1), go);
                    }
                    __builtin_amdgcn_wave_barrier();
                    q_head = 0;
                    q_count = 0;
                }
            }
            walked_pts += __builtin_amdgcn_readfirstlane(sh.walked);
            walked_chunks += nlive;
            __syncthreads();   // the next batch's prologue overwrites the chunk data
        }
        // ---------------------------------------------------------------- reduction of the tile
        // lanes -> wave -> tile: FP64 except kN32, which stays FP32 end to end
        if constexpr (PREC != kN32 && (NT == kTerms || (CMP && MODE == kEval))) {
            // the 28 terms in one transposed butterfly (value k ends on lanes 2k, 2k + 1);
            // the compacted evaluate sums its one term the same way, so its e equals
            // linearize's
            double v[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) v[k] = k < NT ? acc.get64(k) : 0.0;
            const double w = wave_sum_transposed(v, lane);
            if ((lane & 1) == 0 && (lane >> 1) < NT) s_red[wave][lane >> 1] = w;
        } else {
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                if constexpr (PREC == kN32) {
                    const float v = wave_sum(acc.get(k));
                    if (lane == 0) s_red[wave][k] = (double)v;
                } else {
                    const double v = wave_sum(acc.get64(k));
                    if (lane == 0) s_red[wave][k] = v;
                }
            }
        }
        if constexpr (MODE != kBwd) {
#pragma unroll
            for (int l = 0; l < kMaxLevels; ++l) {
                const int32_t v = CMP ? (int32_t)((inl2[l >> 1] >> (16 * (l & 1))) & 0xFFFFu) : wave_sum(inl[l]);
                const int32_t p = CMP ? (int32_t)((prb2[l >> 1] >> (16 * (l & 1))) & 0xFFFFu) : wave_sum(prb[l]);
                if (lane == 0) {
                    s_red[wave][kRowInl + l] = (double)v;
                    s_red[wave][kRowProbe + l] = (double)p;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < kRow) {
            const int k = threadIdx.x;
            double s = 0.0;
            const bool inl_or_probe = (k >= kRowInl && k < kRowWalk) || (k >= kRowProbe && k < kRowChunks);
            if (k == kRowWalk) {
                s = (double)walked_pts;
            } else if (k == kRowChunks) {
                s = (double)walked_chunks;
            } else if (k >= kRowChunks + 1) {
                s = 0.0;
            } else if (PREC == kN32 && k < kTerms) {
                float sf = 0.f;
                for (int w = 0; w < NW; ++w) sf += (float)s_red[w][k];
                s = (double)sf;
            } else {
                for (int w = 0; w < NW; ++w) s += s_red[w][k];
            }
            const bool used = (k < NT) || (MODE != kBwd && inl_or_probe) || k == kRowWalk || k == kRowChunks;
            partials[(int64_t)t * kRow + k] = used ? s : 0.0;
        }
        __syncthreads();
    }
}

// Per-factor reduction of tile rows in tile order (FP64; FP32 for kN32) and the
// frame change H = G^T Bd^T H'' Bd G, b = G^T Bd^T b''.  One 64-thread block per
// factor.  Block 0 also re-arms the tile counter for the next launch.
template <int MODE, int PREC>
__global__ __launch_bounds__(64) void k_reduce(const FactorDesc* __restrict__ fac, const int32_t* __restrict__ tile_first,
                                               int32_t f0, const double* __restrict__ partials,
                                               const double* __restrict__ poses, double* __restrict__ out,
                                               int64_t* __restrict__ inliers, uint32_t* __restrict__ counter,
                                               const double* __restrict__ grad_e, const double* __restrict__ jr,
                                               double* __restrict__ grad_xi, int64_t* __restrict__ work) {
    __shared__ double s[kRow];
    const int f = f0 + blockIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < kParts) counter[threadIdx.x] = 0u;
    const int k = threadIdx.x;
    if (k < kRow) {
        const int32_t a = tile_first[f], bnd = tile_first[f + 1];
        // rows are summed in tile order; each step has kStep row loads in flight
        // before its adds (a factor of a few large sources has hundreds of rows)
        constexpr int kStep = 16;
        if constexpr (PREC == kN32) {
            float sf = 0.f;
            double si = 0.0;
            int32_t t = a;
            for (; t + kStep <= bnd; t += kStep) {
                double v[kStep];
#pragma unroll
                for (int u = 0; u < kStep; ++u) v[u] = partials[(int64_t)(t + u) * kRow + k];
#pragma unroll
                for (int u = 0; u < kStep; ++u) {
                    sf += (float)v[u];
                    si += v[u];
                }
            }
            for (; t < bnd; ++t) {
                const double v = partials[(int64_t)t * kRow + k];
                sf += (float)v;
                si += v;
            }
            s[k] = (k >= kTerms) ? si : (double)sf;   // counts are exact integers in FP64
        } else {
            double acc = 0.0;
            int32_t t = a;
            for (; t + kStep <= bnd; t += kStep) {
                double v[kStep];
#pragma unroll
                for (int u = 0; u < kStep; ++u) v[u] = partials[(int64_t)(t + u) * kRow + k];
#pragma unroll
                for (int u = 0; u < kStep; ++u) acc += v[u];
            }
            for (; t < bnd; ++t) acc += partials[(int64_t)t * kRow + k];
            s[k] = acc;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const FactorDesc& F = fac[f];
    const double* P = poses + 12 * f;
    const double* R = P;
    if (work != nullptr && MODE != kBwd) {
        int64_t* wr = work + (int64_t)kWork * f;
        wr[0] = (int64_t)s[kRowWalk];
        wr[1] = (int64_t)s[kRowChunks];
        for (int l = 0; l < kMaxLevels; ++l) wr[2 + l] = (int64_t)s[kRowProbe + l];
        wr[6] = 0;
        wr[7] = 0;
    }
    const double o[3] = {PREC == kC32 ? F.src_origin[0] : 0.0, PREC == kC32 ? F.src_origin[1] : 0.0,
                         PREC == kC32 ? F.src_origin[2] : 0.0};
    if constexpr (MODE == kEval) {
        out[f] = s[0];
        return;
    }
    if constexpr (MODE == kCount) {
        // overlap rate: fraction of the source points that fall in an occupied voxel
        for (int l = 0; l < F.L; ++l) out[(int64_t)F.L * f + l] = F.n > 0 ? s[kTerms + l] / (double)F.n : 0.0;
        return;
    }
    if constexpr (MODE == kBwd) {
        // g' = Bd^T g'' (rotate both halves back to the source frame), g = G^T g'
        double gw[3], gv[3], g[6];
        for (int i = 0; i < 3; ++i) {
            gw[i] = R[i] * s[0] + R[3 + i] * s[1] + R[6 + i] * s[2];
            gv[i] = R[i] * s[3] + R[3 + i] * s[4] + R[6 + i] * s[5];
        }
        g[0] = gw[0] + (o[1] * gv[2] - o[2] * gv[1]);
        g[1] = gw[1] + (o[2] * gv[0] - o[0] * gv[2]);
        g[2] = gw[2] + (o[0] * gv[1] - o[1] * gv[0]);
        g[3] = gv[0];
        g[4] = gv[1];
        g[5] = gv[2];
        const double ge = grad_e[f];
        for (int i = 0; i < 6; ++i) {
            double v = g[i];
            if (jr != nullptr) {
                v = 0.0;
                for (int j = 0; j < 6; ++j) v += jr[36 * (int64_t)f + 6 * j + i] * g[j];
            }
            grad_xi[6 * (int64_t)f + i] = ge * v;
        }
        return;
    }
    // unpack H'' (symmetric) and b''
    double Hs[36];
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            Hs[6 * i + j] = s[1 + tri(i, j)];
            Hs[6 * j + i] = s[1 + tri(i, j)];
        }
    // M = Bd G (6x6): [[R, 0], [-R (o)x, R]]
    double M[36] = {0};
    double Ox[9] = {0, -o[2], o[1], o[2], 0, -o[0], -o[1], o[0], 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            M[6 * i + j] = R[3 * i + j];
            M[6 * (3 + i) + 3 + j] = R[3 * i + j];
            double ro = 0.0;
            for (int q = 0; q < 3; ++q) ro += R[3 * i + q] * Ox[3 * q + j];
            M[6 * (3 + i) + j] = -ro;
        }
    double HM[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double acc = 0.0;
            for (int q = 0; q < 6; ++q) acc += Hs[6 * i + q] * M[6 * q + j];
            HM[6 * i + j] = acc;
        }
    double* o_row = out + (int64_t)kOutRow * f;
    o_row[0] = s[0];
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            double acc = 0.0;
            for (int q = 0; q < 6; ++q) acc += M[6 * q + i] * HM[6 * q + j];
            o_row[1 + 6 * i + j] = acc;
            o_row[1 + 6 * j + i] = acc;
        }
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
        for (int q = 0; q < 6; ++q) acc += M[6 * q + i] * s[22 + q];
        o_row[37 + i] = acc;
    }
    if (inliers != nullptr)
        for (int l = 0; l < F.L; ++l) inliers[(int64_t)F.L * f + l] = (int64_t)s[kTerms + l];
}

// Correspondences of one factor (keys and found flags in caller order).
template <int PREC>
__global__ void k_correspondences(const FactorDesc* __restrict__ fac, int64_t factor, const double* __restrict__ pose,
                                  int32_t validate, int64_t* __restrict__ keys, int32_t* __restrict__ found) {
    using T = typename PT<PREC>::T;
    const FactorDesc& F = fac[factor];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F.n) return;
    const double* P = pose;
    const int L = F.L;
    const int64_t row = F.perm[i];
    double cs[3] = {0, 0, 0};
    if (validate) {
        const double dc0 = F.viewpoint[0] - P[9], dc1 = F.viewpoint[1] - P[10], dc2 = F.viewpoint[2] - P[11];
        for (int a = 0; a < 3; ++a) cs[a] = P[a] * dc0 + P[3 + a] * dc1 + P[6 + a] * dc2;
    }
    T R[9], tt[3];
    T yl[3];
    for (int k = 0; k < 9; ++k) R[k] = (T)P[k];
    for (int k = 0; k < 3; ++k) tt[k] = (T)P[9 + k];
    bool vis = true;
    int32_t kb[3] = {0, 0, 0};
    const int64_t n_pad = F.n_pad;
    if constexpr (PREC == kC32) {
        const LevelDesc& top = F.lv[L - 1];
        const int64_t c = i / kChunk;
        const double* a = F.anchor + 3 * c;
        const float dx = F.dxyz[i], dy = F.dxyz[n_pad + i], dz = F.dxyz[2 * n_pad + i];
        const double av[3] = {a[0], a[1], a[2]};
        for (int q = 0; q < 3; ++q) {
            double fr;
            anchor_split(P, av, q, top.r64, top.inv_r64, top.K0[q], &fr, &kb[q]);
            yl[q] = chunk_pos32((float)fr, R[3 * q], R[3 * q + 1], R[3 * q + 2], dx, dy, dz);
        }
        if (validate) {
            const float s = ((float)(a[0] - cs[0]) + dx) * F.nrm[i] + ((float)(a[1] - cs[1]) + dy) * F.nrm[n_pad + i] +
                            ((float)(a[2] - cs[2]) + dz) * F.nrm[2 * n_pad + i];
            vis = !(s > 0.0f);
        }
    } else if constexpr (PREC == kN32) {
        const float x0 = F.axyz[i], x1 = F.axyz[n_pad + i], x2 = F.axyz[2 * n_pad + i];
        for (int q = 0; q < 3; ++q) yl[q] = (R[3 * q] * x0 + R[3 * q + 1] * x1 + R[3 * q + 2] * x2) + tt[q];
        if (validate) {
            const float s = (x0 - (float)cs[0]) * F.nrm[i] + (x1 - (float)cs[1]) * F.nrm[n_pad + i] +
                            (x2 - (float)cs[2]) * F.nrm[2 * n_pad + i];
            vis = !(s > 0.0f);
        }
    } else {
        const double x0 = F.xyz64[i], x1 = F.xyz64[n_pad + i], x2 = F.xyz64[2 * n_pad + i];
        for (int q = 0; q < 3; ++q) yl[q] = (R[3 * q] * x0 + R[3 * q + 1] * x1 + R[3 * q + 2] * x2) + tt[q];
        if (validate) {
            const double s = (x0 - cs[0]) * F.nrm64[i] + (x1 - cs[1]) * F.nrm64[n_pad + i] +
                             (x2 - cs[2]) * F.nrm64[2 * n_pad + i];
            vis = !(s > 0.0);
        }
    }
    for (int l = 0; l < L; ++l) {
        const LevelDesc& lv = F.lv[l];
        int64_t kq[3];
        for (int q = 0; q < 3; ++q) {
            if constexpr (PREC == kC32) {
                kq[q] = (int64_t)kb[q] * lv.scale + (int64_t)floor_i32(yl[q] * lv.inv_r);
            } else if constexpr (PREC == kN32) {
                kq[q] = (int64_t)floorf(yl[q] * lv.inv_r) - lv.K0[q];
            } else {
                kq[q] = (int64_t)floor(yl[q] * lv.inv_r64) - lv.K0[q];
            }
            keys[(row * L + l) * 3 + q] = kq[q] + lv.K0[q];
        }
        int32_t fnd;
        if (!vis) fnd = -1;
        else if (!(key_in_range(kq[0]) && key_in_range(kq[1]) && key_in_range(kq[2]))) fnd = 0;
        else fnd = lookup(lv.slots, lv.log2cap, (int32_t)kq[0], (int32_t)kq[1], (int32_t)kq[2]) >= 0 ? 1 : 0;
        found[row * L + l] = fnd;
    }
}

__global__ void k_fill_zero(uint32_t* p, int64_t n_words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_words) p[i] = 0u;
}

// ---------------------------------------------------------------- host launchers

template <int MODE, int PREC, bool KH, bool VAL, int LM>
static vg_status launch_tiles_v(vg_batch* b, const Workspace& ws, const double* d_poses, int32_t t0, int32_t t1,
                                int grid, const double* d_grad_e, void* d_grad_points, int points_dtype) {
    hipStream_t st = b->ctx->stream;
#define VG_LAUNCH(BS)                                                                                          \
    k_tiles<MODE, PREC, BS, KH, VAL, LM><<<grid, BS, 0, st>>>(b->d_fac, b->d_tiles, t0, t1, d_poses, ws.posef, \
                                                              ws.partials, ws.counter, d_grad_e,              \
                                                              d_grad_points, b->d_gslab, points_dtype,        \
                                                              b->tile_order == 2 ? 1 : 0)
    switch (b->block) {
        case 64: VG_LAUNCH(64); break;
        case 128: VG_LAUNCH(128); break;
        case 512: VG_LAUNCH(512); break;
        default: VG_LAUNCH(256); break;
    }
#undef VG_LAUNCH
    VG_HIP(hipGetLastError());
    return VG_OK;
}

template <int MODE, int PREC, bool KH>
static vg_status launch_tiles_t(vg_batch* b, const Workspace& ws, const double* d_poses, int32_t t0, int32_t t1,
                                int grid, const double* d_grad_e, void* d_grad_points, int points_dtype) {
    if (b->opt.surface_validation)
        return launch_tiles_v<MODE, PREC, KH, true, kMaxLevels>(b, ws, d_poses, t0, t1, grid, d_grad_e,
                                                                d_grad_points, points_dtype);
    // single-level compensated batches without validation (the submap factors)
    // get a kernel compiled for one level
    if constexpr (PREC == kC32 && !KH) {
        if (b->L == 1)
            return launch_tiles_v<MODE, PREC, KH, false, 1>(b, ws, d_poses, t0, t1, grid, d_grad_e, d_grad_points,
                                                            points_dtype);
    }
    return launch_tiles_v<MODE, PREC, KH, false, kMaxLevels>(b, ws, d_poses, t0, t1, grid, d_grad_e,
                                                             d_grad_points, points_dtype);
}

vg_status launch_tiles(vg_batch* b, const Workspace& ws, int mode, const double* d_poses, int32_t t0, int32_t t1,
                       int grid, const double* d_grad_e, void* d_grad_points, int points_dtype, int64_t f0,
                       int64_t f1) {
    if (grid < 1) grid = 1;
    if (t1 <= t0) return VG_OK;
    // FP32 pose copies for the FP32 kernels; the one-level compensated kernels
    // (linearize, evaluate, backward) form their rotation from the FP64 poses
    // and read none
    const bool one_level_cmp = mode != kCount && b->opt.precision == kC32 && !b->opt.lane_kahan &&
                               !b->opt.surface_validation && b->L == 1;
    if (b->opt.precision != kF64 && f1 > f0 && !one_level_cmp) {
        const int64_t nf = (f1 - f0) * 16;
        k_stage_poses<<<(int)((nf + 255) / 256), 256, 0, b->ctx->stream>>>(f1 - f0, d_poses + 12 * f0,
                                                                          ws.posef + 16 * f0);
        VG_HIP(hipGetLastError());
    }
    const int p = b->opt.precision;
    const bool kh = b->opt.lane_kahan != 0;
#define VG_DISPATCH(M)                                                                                  \
    if (p == kC32 && kh)                                                                                \
        return launch_tiles_t<M, kC32, true>(b, ws, d_poses, t0, t1, grid, d_grad_e, d_grad_points, points_dtype); \
    if (p == kC32)                                                                                      \
        return launch_tiles_t<M, kC32, false>(b, ws, d_poses, t0, t1, grid, d_grad_e, d_grad_points, points_dtype); \
    if (p == kN32)                                                                                      \
        return launch_tiles_t<M, kN32, false>(b, ws, d_poses, t0, t1, grid, d_grad_e, d_grad_points, points_dtype); \
    return launch_tiles_t<M, kF64, false>(b, ws, d_poses, t0, t1, grid, d_grad_e, d_grad_points, points_dtype);
    if (mode == kLin) { VG_DISPATCH(kLin) }
    if (mode == kEval) { VG_DISPATCH(kEval) }
    if (mode == kCount) { VG_DISPATCH(kCount) }
    VG_DISPATCH(kBwd)
#undef VG_DISPATCH
}

template <int MODE, int PREC>
static void reduce_t(vg_batch* b, const Workspace& ws, const double* d_poses, int32_t f0, int32_t f1, double* d_out,
                     int64_t* d_inl, const double* d_grad_e, const double* d_jr, double* d_grad_xi) {
    k_reduce<MODE, PREC><<<f1 - f0, 64, 0, b->ctx->stream>>>(b->d_fac, b->d_tile_first, f0, ws.partials, d_poses,
                                                             d_out, d_inl, ws.counter, d_grad_e, d_jr, d_grad_xi,
                                                             ws.work);
}

vg_status launch_reduce(vg_batch* b, const Workspace& ws, int mode, const double* d_poses, int32_t f0, int32_t f1,
                        double* d_out, int64_t* d_inliers, const double* d_grad_e, const double* d_jr,
                        double* d_grad_xi) {
    if (f1 <= f0) return VG_OK;
    const int p = b->opt.precision;
#define VG_R(M)                                                                               \
    if (p == kC32) reduce_t<M, kC32>(b, ws, d_poses, f0, f1, d_out, d_inliers, d_grad_e, d_jr, d_grad_xi); \
    else if (p == kN32) reduce_t<M, kN32>(b, ws, d_poses, f0, f1, d_out, d_inliers, d_grad_e, d_jr, d_grad_xi); \
    else reduce_t<M, kF64>(b, ws, d_poses, f0, f1, d_out, d_inliers, d_grad_e, d_jr, d_grad_xi);
    if (mode == kLin) { VG_R(kLin) }
    else if (mode == kEval) { VG_R(kEval) }
    else if (mode == kCount) { VG_R(kCount) }
    else { VG_R(kBwd) }
#undef VG_R
    VG_HIP(hipGetLastError());
    return VG_OK;
}

vg_status launch_grad_combine(vg_batch* b, void* d_grad_points, int points_dtype) {
    if (b->shared_rows == 0 || d_grad_points == nullptr) return VG_OK;
    const int grid = (int)((b->shared_rows + 255) / 256);
    k_grad_combine<<<grid, 256, 0, b->ctx->stream>>>(b->d_shared, (int32_t)b->h_shared.size(), b->shared_rows,
                                                     b->d_slab_off, b->d_gslab, d_grad_points, points_dtype);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

vg_status launch_correspondences(vg_batch* b, const double* d_pose, int64_t factor, int64_t* d_keys,
                                 int32_t* d_found) {
    const int64_t n = b->h_fac[factor].n;
    if (n == 0) return VG_OK;
    const int grid = (int)((n + 255) / 256);
    const int v = b->opt.surface_validation;
    hipStream_t st = b->ctx->stream;
    if (b->opt.precision == kC32)
        k_correspondences<kC32><<<grid, 256, 0, st>>>(b->d_fac, factor, d_pose, v, d_keys, d_found);
    else if (b->opt.precision == kN32)
        k_correspondences<kN32><<<grid, 256, 0, st>>>(b->d_fac, factor, d_pose, v, d_keys, d_found);
    else
        k_correspondences<kF64><<<grid, 256, 0, st>>>(b->d_fac, factor, d_pose, v, d_keys, d_found);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

vg_status launch_zero(vg_context* ctx, void* d_ptr, size_t bytes) {
    if (bytes == 0) return VG_OK;
    const int64_t words = (int64_t)((bytes + 3) / 4);
    const int grid = (int)((words + 255) / 256);
    k_fill_zero<<<grid, 256, 0, ctx->stream>>>((uint32_t*)d_ptr, words);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

}  // namespace vg
