// Frame preprocessing (GLIM Sec. IV-A; Sec. III-C, Preprocessing): voxel-grid
// downsampling, exact k-nearest-neighbour search and neighbour covariances with
// plane-to-plane regularisation and oriented normals.
//
// Device pipeline:
//   1. FP64 voxel keys -> stable radix sort of (key, point) -> run-length
//      encoding; one thread per voxel sums its run in input order (FP64).
//   2. k-NN on a hierarchy of uniform grids (cells of 2r, 4r, ..., 64r):
//      per grid, points sorted by cell and cells in an open-addressing table.
//      One thread per query walks cubic shells of cells around its own cell
//      (radius 0..1 cells) and keeps the k best (distance, index) pairs in
//      registers, candidates read four at a time and rejected against the
//      current k-th pair before any insertion work; the walk stops once the k-th distance is below the
//      distance to the unvisited region (strictly, with a 1e-9 relative
//      margin), so the result is exact.  A query that is not settled within
//      two shells starts again on the next coarser grid (sparse regions: few
//      large cells instead of many empty small ones); on the coarsest grid it
//      walks on until settled, or scans every point once the next shell would
//      hold more cells than the grid has occupied cells.
//   3. one thread per point: mean and covariance of its neighbours (FP64),
//      cyclic Jacobi eigen-decomposition, normal = smallest eigenvector,
//      oriented towards the sensor, C = I - (1 - 1e-3) n n^T.
#include <hipcub/hipcub.hpp>

#include <climits>
#include <cmath>
#include <vector>

#include "vg_device.h"

namespace vg {
namespace {

constexpr int kPBits = 21;                       // bits per axis of a packed preprocessing key
constexpr int64_t kPBias = 1ll << (kPBits - 1);  // keys live in [-2^20, 2^20)
constexpr uint64_t kPEmpty = ~0ull;
constexpr double kEpsReg = 1e-3;
constexpr int kMaxK = 32;

__device__ __forceinline__ bool pkey_ok(int64_t q) { return q >= -kPBias && q < kPBias; }

// lexicographic (x, y, z) order of the packed key equals the order of the integer triple
__device__ __forceinline__ uint64_t pack21(int64_t x, int64_t y, int64_t z) {
    return ((uint64_t)(x + kPBias) << (2 * kPBits)) | ((uint64_t)(y + kPBias) << kPBits) | (uint64_t)(z + kPBias);
}

__device__ __forceinline__ void unpack21(uint64_t k, int64_t* x, int64_t* y, int64_t* z) {
    const uint64_t m = (1ull << kPBits) - 1;
    *x = (int64_t)((k >> (2 * kPBits)) & m) - kPBias;
    *y = (int64_t)((k >> kPBits) & m) - kPBias;
    *z = (int64_t)(k & m) - kPBias;
}

__device__ __forceinline__ uint32_t cell_slot(uint64_t key, uint32_t lg) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - lg));
}

__global__ void k_ds_keys(const double* __restrict__ xyz, int64_t n, double r, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ idx, int32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double qx = floor(xyz[3 * i + 0] / r);
    const double qy = floor(xyz[3 * i + 1] / r);
    const double qz = floor(xyz[3 * i + 2] / r);
    const double lim = (double)kPBias;
    if (!(qx >= -lim && qx < lim && qy >= -lim && qy < lim && qz >= -lim && qz < lim)) {
        atomicOr(flag, 1);
        keys[i] = 0;
    } else {
        keys[i] = pack21((int64_t)qx, (int64_t)qy, (int64_t)qz);
    }
    idx[i] = (int32_t)i;
}

// one thread per voxel: FP64 sum of its run (input order), then the mean; the
// point's grid cell for the neighbour search
__global__ void k_ds_centroids(const double* __restrict__ xyz, const int32_t* __restrict__ sorted_idx,
                               const int32_t* __restrict__ offsets, const int32_t* __restrict__ counts, int64_t m,
                               double* __restrict__ out, int32_t* __restrict__ out_counts) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m) return;
    const int32_t o = offsets[v], c = counts[v];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t j = 0; j < c; ++j) {
        const int32_t p = sorted_idx[o + j];
        sx += xyz[3 * p + 0];
        sy += xyz[3 * p + 1];
        sz += xyz[3 * p + 2];
    }
    const double cx = sx / (double)c, cy = sy / (double)c, cz = sz / (double)c;
    out[3 * v + 0] = cx;
    out[3 * v + 1] = cy;
    out[3 * v + 2] = cz;
    out_counts[v] = c;
}

// grid cell of every downsampled point (cell size h >= 2r: |c / h| < 2^19, always
// packable) and the grid's cell bounding box
__global__ void k_grid_keys(const double* __restrict__ c, int64_t m, double h, uint64_t* __restrict__ cell_keys,
                            int32_t* __restrict__ cell_idx, int32_t* __restrict__ box) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    if (v < m) {
        const int64_t gx = (int64_t)floor(c[3 * v] / h), gy = (int64_t)floor(c[3 * v + 1] / h),
                      gz = (int64_t)floor(c[3 * v + 2] / h);
        cell_keys[v] = pack21(gx, gy, gz);
        cell_idx[v] = (int32_t)v;
        lo[0] = hi[0] = (int32_t)gx;
        lo[1] = hi[1] = (int32_t)gy;
        lo[2] = hi[2] = (int32_t)gz;
    }
    // the wave's box first, then one atomic per wave and bound
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], w));
            hi[a] = max(hi[a], __shfl_xor(hi[a], w));
        }
    if ((threadIdx.x & 63) == 0 && lo[0] <= hi[0]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(&box[a], lo[a]);
            atomicMax(&box[3 + a], hi[a]);
        }
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64p(uint64_t* p, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_cells_insert(const uint64_t* __restrict__ ucells, const int32_t* __restrict__ nc,
                               uint64_t* __restrict__ hkeys, int32_t* __restrict__ hval, uint32_t lg) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= *nc) return;
    const uint64_t key = ucells[c];
    const uint32_t mask = (1u << lg) - 1;
    uint32_t s = cell_slot(key, lg);
    for (;;) {
        const unsigned long long prev =
            atomicCAS((unsigned long long*)&hkeys[s], (unsigned long long)kPEmpty, (unsigned long long)key);
        if (prev == kPEmpty || prev == key) {
            hval[s] = (int32_t)c;
            return;
        }
        s = (s + 1) & mask;
    }
}

// coordinates in cell order (SoA) so that a cell's points are contiguous
__global__ void k_cells_gather(const double* __restrict__ xyz, const int32_t* __restrict__ cidx, int64_t m,
                               double* __restrict__ sx, double* __restrict__ sy, double* __restrict__ sz) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int32_t i = cidx[t];
    sx[t] = xyz[3 * i + 0];
    sy[t] = xyz[3 * i + 1];
    sz[t] = xyz[3 * i + 2];
}

__device__ __forceinline__ int32_t cell_find(const uint64_t* __restrict__ hkeys, const int32_t* __restrict__ hval,
                                             uint32_t lg, uint64_t key) {
    const uint32_t mask = (1u << lg) - 1;
    uint32_t s = cell_slot(key, lg);
    for (;;) {
        const uint64_t k = hkeys[s];
        if (k == key) return hval[s];
        if (k == kPEmpty) return -1;
        s = (s + 1) & mask;
    }
}

// squared distance with every operation rounded on its own: this file is
// compiled with -ffp-contract=off, so no multiply-add is fused
__device__ __forceinline__ double sqdist_rn(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = bx - ax, dy = by - ay, dz = bz - az;
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    return (xx + yy) + zz;
}

__device__ __forceinline__ bool pair_less(double d, int32_t j, double D, int32_t J) {
    return d < D || (d == D && j < J);
}

// Insert (d, j) into the list sorted by (distance, index) whose first kk slots
// are live.  Precondition: (d, j) is below the pair at place kk - 1.  Walking
// down from that place, each slot either takes its upper neighbour (the new
// pair goes further up) or the new pair, once; every slot is written once,
// after the slot below it has been read, so the update is in place.
template <int KMAX>
__device__ __forceinline__ void knn_insert(double (&D)[KMAX], int32_t (&I)[KMAX], int kk, double d, int32_t j) {
    bool placed = false;
#pragma unroll
    for (int s = KMAX - 1; s > 0; --s) {
        if (s < kk && !placed) {
            if (pair_less(d, j, D[s - 1], I[s - 1])) {
                D[s] = D[s - 1];
                I[s] = I[s - 1];
            } else {
                D[s] = d;
                I[s] = j;
                placed = true;
            }
        }
    }
    if (!placed) {
        D[0] = d;
        I[0] = j;
    }
}

// the pair at place kk - 1 (the k-th best so far)
template <int KMAX>
__device__ __forceinline__ void kth_pair(const double (&D)[KMAX], const int32_t (&I)[KMAX], int kk, double& wD,
                                         int32_t& wI) {
    wD = D[0];
    wI = I[0];
#pragma unroll
    for (int s = 1; s < KMAX; ++s)
        if (s == kk - 1) {
            wD = D[s];
            wI = I[s];
        }
}

constexpr int kGrids = 6;       // cell sizes 2r, 4r, ..., 64r
constexpr int kShells = 1;      // shells walked on every grid but the coarsest
constexpr int kBudget = 1024;   // candidates a query may scan before it is handed to the wave-wide pass

struct KnnGrid {
    const double* sx;           // coordinates in cell order
    const double* sy;
    const double* sz;
    const int32_t* cidx;        // cell order -> point index
    const int32_t* cstart;      // per cell (cell ordinal)
    const int32_t* ccount;
    const uint64_t* hkeys;      // cell table
    const int32_t* hval;
    const int32_t* box;         // cell bounding box (6)
    const int32_t* ncells;      // occupied cells (device scalar)
    uint32_t lg;
    double h;
};

struct KnnGrids {
    KnnGrid g[kGrids];
};

// Exact k-NN, one thread per query, queries taken in the finest grid's cell order.
//
// A pass over grid g lists the k best pairs among the points of the cells it
// visits.  If it cannot prove them final, its k-th pair P is still an upper
// bound of the true k-th pair (its points are a subset of the cloud), so the
// next pass (a) starts on the first coarser grid whose cells are at least
// sqrt(d(P)) wide, (b) skips cells whose box lies farther than sqrt(d(P)), and
// (c) keeps only candidates that do not exceed P.  Every point of the true
// k best lies within sqrt(d(P)), so that pass still finds all of them.
template <int KMAX>
__global__ void __launch_bounds__(128) k_knn(const KnnGrid* __restrict__ grids, int64_t m, int k,
                                             int32_t* __restrict__ nbr, double* __restrict__ nd2,
                                             int32_t* __restrict__ hard, int32_t* __restrict__ n_hard) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const double qx = grids[0].sx[t], qy = grids[0].sy[t], qz = grids[0].sz[t];
    const int kk = (int)min((int64_t)k, m);
    double D[KMAX];
    int32_t I[KMAX];
    double bD = INFINITY;   // bound carried between passes: the previous pass's k-th pair
    int32_t bI = INT_MAX;
    bool done = false;
    int64_t scanned = 0;    // candidates read; past kBudget the query goes to the wave-wide pass
#pragma unroll 1
    for (int gi = 0; gi < kGrids && !done; ++gi) {
        const KnnGrid g = grids[gi];
        const double h = g.h;
        const bool last = (gi == kGrids - 1);
        if (!last && bD < INFINITY && h * h <= bD) continue;   // cells too small for the bound
        const int64_t cx = (int64_t)floor(qx / h), cy = (int64_t)floor(qy / h), cz = (int64_t)floor(qz / h);
        const int32_t bx0 = g.box[0], by0 = g.box[1], bz0 = g.box[2], bx1 = g.box[3], by1 = g.box[4],
                      bz1 = g.box[5];
        const int64_t rmax = max(max(max(cx - bx0, bx1 - cx), max(cy - by0, by1 - cy)), max(cz - bz0, bz1 - cz));
        const int64_t nc = *g.ncells;
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            D[s] = INFINITY;
            I[s] = INT_MAX;
        }
        // threshold: a candidate is kept iff it does not exceed (wD, wI); while the
        // list is not full that is the carried bound, then the list's k-th pair
        double wD = bD;
        int32_t wI = bI;
        int filled = 0;
        for (int64_t r = 0;; ++r) {
            if (!last && r > kShells) break;                       // not settled: next grid
            if (last && r > 0 && (2 * r + 1) * (2 * r + 1) * (2 * r + 1) > 4 * nc + 64) goto handover;
            for (int64_t dx = -r; dx <= r; ++dx) {
                const int64_t x = cx + dx;
                if (x < bx0 || x > bx1) continue;
                const double ex = fmax(0.0, fmax((double)x * h - qx, qx - (double)(x + 1) * h));
                for (int64_t dy = -r; dy <= r; ++dy) {
                    const int64_t y = cy + dy;
                    if (y < by0 || y > by1) continue;
                    const double ey = fmax(0.0, fmax((double)y * h - qy, qy - (double)(y + 1) * h));
                    const bool edge = (dx == -r || dx == r || dy == -r || dy == r);
                    const int64_t step = (edge || r == 0) ? 1 : 2 * r;
                    for (int64_t dz = -r; dz <= r; dz += step) {
                        const int64_t z = cz + dz;
                        if (z < bz0 || z > bz1) continue;
                        const double ez = fmax(0.0, fmax((double)z * h - qz, qz - (double)(z + 1) * h));
                        // the cell's box is farther than the threshold: nothing in it can be kept
                        // (margin for the rounding of the box and of the distances)
                        if ((ex * ex + ey * ey + ez * ez) * (1.0 - 1e-9) > wD) continue;
                        const int32_t c = cell_find(g.hkeys, g.hval, g.lg, pack21(x, y, z));
                        if (c < 0) continue;
                        const int32_t p0 = g.cstart[c], p1 = p0 + g.ccount[c];
                        scanned += p1 - p0;
                        if (scanned > kBudget) goto handover;
                        for (int32_t p = p0; p < p1; ++p) {
                            const double d = sqdist_rn(qx, qy, qz, g.sx[p], g.sy[p], g.sz[p]);
                            const int32_t j = g.cidx[p];
                            if (!pair_less(wD, wI, d, j)) {   // (d, j) <= threshold
                                knn_insert<KMAX>(D, I, kk, d, j);
                                if (++filled >= kk) kth_pair<KMAX>(D, I, kk, wD, wI);
                            }
                        }
                    }
                }
            }
            if (r >= rmax) {   // every occupied cell of this grid visited
                done = true;
                break;
            }
            if (filled >= kk) {
                const double bx = fmin(qx - (double)(cx - r) * h, (double)(cx + r + 1) * h - qx);
                const double by = fmin(qy - (double)(cy - r) * h, (double)(cy + r + 1) * h - qy);
                const double bz = fmin(qz - (double)(cz - r) * h, (double)(cz + r + 1) * h - qz);
                const double b = fmin(bx, fmin(by, bz));
                if (b > 0.0 && wD < b * b * (1.0 - 1e-9)) {
                    done = true;
                    break;
                }
            }
        }
        if (!done && filled >= kk) {
            bD = wD;
            bI = wI;
        }
    }
    {
        const int32_t i = grids[0].cidx[t];
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            if (s < k) {
                const bool ok = s < kk;
                nbr[(int64_t)i * k + s] = ok ? I[s] : -1;
                nd2[(int64_t)i * k + s] = ok ? D[s] : INFINITY;
            }
        }
        return;
    }
handover:
    hard[atomicAdd(n_hard, 1)] = (int32_t)t;
}

// The queries the grid walk handed over: one wave per query scans every point
// (each lane a strided share, its own k best in registers), then the lanes'
// lists are merged by k rounds of a wave-wide minimum over their heads.
template <int KMAX>
__global__ void __launch_bounds__(64) k_knn_wave(const KnnGrid* __restrict__ grids, int64_t m, int k,
                                                 const int32_t* __restrict__ hard, const int32_t* __restrict__ n_hard,
                                                 uint32_t* __restrict__ next, int32_t* __restrict__ nbr,
                                                 double* __restrict__ nd2) {
    const KnnGrid g = grids[0];
    const int lane = threadIdx.x;
    const int kk = (int)min((int64_t)k, m);
    for (;;) {
        int32_t q = 0;
        if (lane == 0) q = (int32_t)atomicAdd(next, 1u);
        q = __shfl(q, 0);
        if (q >= *n_hard) break;
        const int32_t t = hard[q];
        const double qx = g.sx[t], qy = g.sy[t], qz = g.sz[t];
        double D[KMAX];
        int32_t I[KMAX];
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            D[s] = INFINITY;
            I[s] = INT_MAX;
        }
        double wD = INFINITY;
        int32_t wI = INT_MAX;
        int filled = 0;
        for (int64_t p = lane; p < m; p += 64) {
            const double d = sqdist_rn(qx, qy, qz, g.sx[p], g.sy[p], g.sz[p]);
            const int32_t j = g.cidx[p];
            if (!pair_less(wD, wI, d, j)) {
                knn_insert<KMAX>(D, I, kk, d, j);
                if (++filled >= kk) kth_pair<KMAX>(D, I, kk, wD, wI);
            }
        }
        const int32_t i = g.cidx[t];
        for (int o = 0; o < kk; ++o) {
            double bd = D[0];
            int32_t bj = I[0];
#pragma unroll
            for (int w = 32; w >= 1; w >>= 1) {
                const double od = __shfl_xor(bd, w);
                const int32_t oj = __shfl_xor(bj, w);
                if (pair_less(od, oj, bd, bj)) {
                    bd = od;
                    bj = oj;
                }
            }
            if (D[0] == bd && I[0] == bj) {   // this lane's head won: drop it
#pragma unroll
                for (int s = 0; s + 1 < KMAX; ++s) {
                    D[s] = D[s + 1];
                    I[s] = I[s + 1];
                }
                D[KMAX - 1] = INFINITY;
                I[KMAX - 1] = INT_MAX;
            }
            if (lane == 0) {
                nbr[(int64_t)i * k + o] = bj;
                nd2[(int64_t)i * k + o] = bd;
            }
        }
        if (lane == 0)
            for (int o = kk; o < k; ++o) {
                nbr[(int64_t)i * k + o] = -1;
                nd2[(int64_t)i * k + o] = INFINITY;
            }
    }
}

// One Jacobi rotation in the (p, q) plane: annihilates a[p][q] (Golub & Van Loan,
// symmetric Schur decomposition), accumulates the rotation into v.
template <int P, int Q, int R>
__device__ __forceinline__ void jacobi_rot(double (&a)[3][3], double (&v)[3][3]) {
    const double apq = a[P][Q];
    if (apq == 0.0) return;
    const double tau = (a[Q][Q] - a[P][P]) / (2.0 * apq);
    double t;
    if (fabs(tau) > 1e150) {
        t = 0.5 / tau;
    } else {
        t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    }
    const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
    a[P][P] -= t * apq;
    a[Q][Q] += t * apq;
    a[P][Q] = a[Q][P] = 0.0;
    const double arp = a[R][P], arq = a[R][Q];
    a[R][P] = a[P][R] = c * arp - s * arq;
    a[R][Q] = a[Q][R] = s * arp + c * arq;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double vp = v[i][P], vq = v[i][Q];
        v[i][P] = c * vp - s * vq;
        v[i][Q] = s * vp + c * vq;
    }
}

__global__ void k_cov_normals(const double* __restrict__ xyz, const int32_t* __restrict__ nbr, int64_t m, int k,
                              double ox, double oy, double oz, double* __restrict__ cov,
                              double* __restrict__ cov_raw, double* __restrict__ nrm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t* row = nbr + i * k;
    int kk = 0;
    double mx = 0.0, my = 0.0, mz = 0.0;
    for (int s = 0; s < k; ++s) {
        const int32_t j = row[s];
        if (j < 0) break;
        mx += xyz[3 * j + 0];
        my += xyz[3 * j + 1];
        mz += xyz[3 * j + 2];
        ++kk;
    }
    const double inv = 1.0 / (double)kk;
    mx *= inv;
    my *= inv;
    mz *= inv;
    double cxx = 0, cxy = 0, cxz = 0, cyy = 0, cyz = 0, czz = 0;
    for (int s = 0; s < kk; ++s) {
        const int32_t j = row[s];
        const double dx = xyz[3 * j + 0] - mx, dy = xyz[3 * j + 1] - my, dz = xyz[3 * j + 2] - mz;
        cxx += dx * dx;
        cxy += dx * dy;
        cxz += dx * dz;
        cyy += dy * dy;
        cyz += dy * dz;
        czz += dz * dz;
    }
    cxx *= inv;
    cxy *= inv;
    cxz *= inv;
    cyy *= inv;
    cyz *= inv;
    czz *= inv;
    double* cr = cov_raw + 6 * i;
    cr[0] = cxx;
    cr[1] = cxy;
    cr[2] = cxz;
    cr[3] = cyy;
    cr[4] = cyz;
    cr[5] = czz;
    double a[3][3] = {{cxx, cxy, cxz}, {cxy, cyy, cyz}, {cxz, cyz, czz}};
    double v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    const double scale = cxx * cxx + cyy * cyy + czz * czz + 2.0 * (cxy * cxy + cxz * cxz + cyz * cyz);
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        if (off == 0.0 || off <= 1e-34 * scale) break;
        jacobi_rot<0, 1, 2>(a, v);
        jacobi_rot<0, 2, 1>(a, v);
        jacobi_rot<1, 2, 0>(a, v);
    }
    // smallest eigenvalue's column (first index on ties)
    int c = 0;
    if (a[1][1] < a[c][c]) c = 1;
    if (a[2][2] < a[c][c]) c = 2;
    double nx = c == 0 ? v[0][0] : (c == 1 ? v[0][1] : v[0][2]);
    double ny = c == 0 ? v[1][0] : (c == 1 ? v[1][1] : v[1][2]);
    double nz = c == 0 ? v[2][0] : (c == 1 ? v[2][1] : v[2][2]);
    const double px = xyz[3 * i + 0], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
    if (nx * (ox - px) + ny * (oy - py) + nz * (oz - pz) < 0.0) {
        nx = -nx;
        ny = -ny;
        nz = -nz;
    }
    double* no = nrm + 3 * i;
    no[0] = nx;
    no[1] = ny;
    no[2] = nz;
    const double w = 1.0 - kEpsReg;
    double* co = cov + 6 * i;
    co[0] = 1.0 - w * nx * nx;
    co[1] = -w * nx * ny;
    co[2] = -w * nx * nz;
    co[3] = 1.0 - w * ny * ny;
    co[4] = -w * ny * nz;
    co[5] = 1.0 - w * nz * nz;
}

int grid_of(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

// Temporaries of one preprocessing call, carved from the context's workspace;
// what does not fit is allocated and freed, and the workspace grows to the
// call's total afterwards, so frames of similar size allocate nothing.
struct Scratch {
    vg_context* ctx;
    size_t off = 0, need = 0;
    std::vector<void*> ptrs;
    explicit Scratch(vg_context* c) : ctx(c) {}
    ~Scratch() {
        (void)hipStreamSynchronize(ctx->stream);   // also on early error returns
        for (void* p : ptrs) (void)hipFree(p);
        if (need > ctx->ws_bytes) {
            if (ctx->ws) (void)hipFree(ctx->ws);
            ctx->ws = nullptr;
            ctx->ws_bytes = 0;
            if (hipMalloc(&ctx->ws, need) == hipSuccess) ctx->ws_bytes = need;
        }
    }
    template <typename T>
    hipError_t get(T** p, size_t count) {
        const size_t bytes = (sizeof(T) * (count ? count : 1) + 255) & ~(size_t)255;
        need += bytes;
        if (ctx->ws && off + bytes <= ctx->ws_bytes) {
            *p = (T*)((char*)ctx->ws + off);
            off += bytes;
            return hipSuccess;
        }
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, bytes);
        if (e == hipSuccess) ptrs.push_back(q);
        *p = (T*)q;
        return e;
    }
};

// every output array of a cloud in one allocation
hipError_t alloc_cloud(vg_cloud* c, int64_t m, int k) {
    const size_t nd = (size_t)m * (3 + 6 + 6 + 3 + k), ni = (size_t)m * (1 + k);
    void* b = nullptr;
    hipError_t e = hipMalloc(&b, sizeof(double) * (nd ? nd : 1) + sizeof(int32_t) * (ni ? ni : 1));
    if (e != hipSuccess) return e;
    c->block = b;
    double* d = (double*)b;
    c->xyz = d;
    c->cov = d + 3 * m;
    c->cov_raw = d + 9 * m;
    c->nrm = d + 15 * m;
    c->d2 = d + 18 * m;
    int32_t* i = (int32_t*)(d + (nd ? nd : 1));
    c->counts = i;
    c->nbr = i + m;
    return hipSuccess;
}

}  // namespace

void free_cloud(vg_cloud* c) {
    if (c->block) (void)hipFree(c->block);
    c->block = nullptr;
    c->xyz = c->cov = c->cov_raw = c->nrm = c->d2 = nullptr;
    c->counts = c->nbr = nullptr;
}

vg_status preprocess_frame(vg_context* ctx, const double* d_xyz, int64_t n, double r, int k, const double sensor[3],
                           vg_cloud* out) {
    hipStream_t st = ctx->stream;
    out->k = k;
    out->m = 0;
    if (n == 0) {
        VG_HIP(alloc_cloud(out, 0, k));
        return VG_OK;
    }
    Scratch sc(ctx);
    int32_t* d_small = nullptr;   // flag, voxel count, hand-over count and cursor
    VG_HIP(sc.get(&d_small, 16));
    // 1. downsampling
    uint64_t *keys, *keys_s, *ukeys;
    int32_t *idx, *idx_s, *counts, *offsets;
    VG_HIP(sc.get(&keys, n));
    VG_HIP(sc.get(&keys_s, n));
    VG_HIP(sc.get(&ukeys, n));
    VG_HIP(sc.get(&idx, n));
    VG_HIP(sc.get(&idx_s, n));
    VG_HIP(sc.get(&counts, n));
    VG_HIP(sc.get(&offsets, n));
    size_t tmp_bytes = 0, b2 = 0, b3 = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys_s, idx, idx_s, (int)n, 0, 3 * kPBits);
    (void)hipcub::DeviceRunLengthEncode::Encode(nullptr, b2, keys_s, ukeys, counts, d_small, (int)n);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b3, counts, offsets, (int)n);
    tmp_bytes = std::max(tmp_bytes, std::max(b2, b3)) + 256;
    void* tmp = nullptr;
    VG_HIP(sc.get((char**)&tmp, tmp_bytes));
    int32_t h_init[16] = {0, 0, 0, 0, 0, 0, 0, 0, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN, 0, 0};
    VG_HIP(hipMemcpyAsync(d_small, h_init, sizeof(h_init), hipMemcpyHostToDevice, st));
    k_ds_keys<<<grid_of(n), 256, 0, st>>>(d_xyz, n, r, keys, idx, d_small);
    VG_HIP(hipGetLastError());
    size_t tb = tmp_bytes;
    VG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys_s, idx, idx_s, (int)n, 0, 3 * kPBits, st));
    tb = tmp_bytes;
    VG_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, keys_s, ukeys, counts, d_small + 1, (int)n, st));
    int32_t h_small[2] = {0, 0};
    VG_HIP(hipMemcpyAsync(h_small, d_small, sizeof(h_small), hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    if (h_small[0]) {
        set_error("downsampling voxel key outside the packable range (|floor(x / r)| >= 2^20 on an axis)");
        return VG_ERR_KEY_RANGE;
    }
    const int64_t m = h_small[1];
    tb = tmp_bytes;
    VG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, counts, offsets, (int)m, st));
    VG_HIP(alloc_cloud(out, m, k));
    out->m = m;
    k_ds_centroids<<<grid_of(m), 256, 0, st>>>(d_xyz, idx_s, offsets, counts, m, out->xyz, out->counts);
    VG_HIP(hipGetLastError());
    // 2. grids of cells and the neighbour search (no host round trip: the cell
    // counts stay on the device, tables are sized for m cells)
    uint32_t lg = 6;
    while ((1ull << lg) < 2ull * (uint64_t)m) ++lg;
    KnnGrids G{};
    int32_t* d_grid_small = nullptr;   // per grid: box (6), cell count, pad
    VG_HIP(sc.get(&d_grid_small, 8 * kGrids));
    {
        std::vector<int32_t> init(8 * kGrids);
        for (int gi = 0; gi < kGrids; ++gi) {
            int32_t* b = init.data() + 8 * gi;
            b[0] = b[1] = b[2] = INT32_MAX;
            b[3] = b[4] = b[5] = INT32_MIN;
            b[6] = b[7] = 0;
        }
        VG_HIP(hipMemcpyAsync(d_grid_small, init.data(), sizeof(int32_t) * init.size(), hipMemcpyHostToDevice, st));
        VG_HIP(hipStreamSynchronize(st));   // init lives on the host stack
    }
    uint64_t *ckeys, *ucells;
    int32_t* cidx;
    VG_HIP(sc.get(&ckeys, m));
    VG_HIP(sc.get(&ucells, m));
    VG_HIP(sc.get(&cidx, m));
    double h = 2.0 * r;
    for (int gi = 0; gi < kGrids; ++gi, h *= 2.0) {
        KnnGrid& g = G.g[gi];
        uint64_t* ckeys_s;
        int32_t *cidx_s, *ccount, *cstart, *hval;
        uint64_t* hkeys;
        double *sx, *sy, *sz;
        VG_HIP(sc.get(&ckeys_s, m));
        VG_HIP(sc.get(&cidx_s, m));
        VG_HIP(sc.get(&ccount, m));
        VG_HIP(sc.get(&cstart, m));
        VG_HIP(sc.get(&hkeys, (size_t)1 << lg));
        VG_HIP(sc.get(&hval, (size_t)1 << lg));
        VG_HIP(sc.get(&sx, m));
        VG_HIP(sc.get(&sy, m));
        VG_HIP(sc.get(&sz, m));
        int32_t* box = d_grid_small + 8 * gi;
        k_grid_keys<<<grid_of(m), 256, 0, st>>>(out->xyz, m, h, ckeys, cidx, box);
        VG_HIP(hipGetLastError());
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, ckeys, ckeys_s, cidx, cidx_s, (int)m, 0, 3 * kPBits, st));
        k_fill_i32<<<grid_of(m), 256, 0, st>>>(ccount, m, 0);
        VG_HIP(hipGetLastError());
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, ckeys_s, ucells, ccount, box + 6, (int)m, st));
        tb = tmp_bytes;
        VG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, ccount, cstart, (int)m, st));
        k_fill_u64p<<<grid_of((int64_t)1 << lg), 256, 0, st>>>(hkeys, (int64_t)1 << lg, kPEmpty);
        VG_HIP(hipGetLastError());
        k_cells_insert<<<grid_of(m), 256, 0, st>>>(ucells, box + 6, hkeys, hval, lg);
        VG_HIP(hipGetLastError());
        k_cells_gather<<<grid_of(m), 256, 0, st>>>(out->xyz, cidx_s, m, sx, sy, sz);
        VG_HIP(hipGetLastError());
        g = KnnGrid{sx, sy, sz, cidx_s, cstart, ccount, hkeys, hval, box, box + 6, lg, h};
    }
    KnnGrid* d_grids = nullptr;
    VG_HIP(sc.get(&d_grids, kGrids));
    VG_HIP(hipMemcpyAsync(d_grids, G.g, sizeof(G.g), hipMemcpyHostToDevice, st));
    int32_t* d_hard = nullptr;
    VG_HIP(sc.get(&d_hard, m));
    int32_t* d_nhard = d_small + 4;                      // zeroed with d_small
    uint32_t* d_next = (uint32_t*)(d_small + 5);
    const int kb = 128;
    const int waves = 2048;
    if (k <= 8) {
        k_knn<8><<<grid_of(m, kb), kb, 0, st>>>(d_grids, m, k, out->nbr, out->d2, d_hard, d_nhard);
        k_knn_wave<8><<<waves, 64, 0, st>>>(d_grids, m, k, d_hard, d_nhard, d_next, out->nbr, out->d2);
    } else if (k <= 16) {
        k_knn<16><<<grid_of(m, kb), kb, 0, st>>>(d_grids, m, k, out->nbr, out->d2, d_hard, d_nhard);
        k_knn_wave<16><<<waves, 64, 0, st>>>(d_grids, m, k, d_hard, d_nhard, d_next, out->nbr, out->d2);
    } else {
        k_knn<32><<<grid_of(m, kb), kb, 0, st>>>(d_grids, m, k, out->nbr, out->d2, d_hard, d_nhard);
        k_knn_wave<32><<<waves, 64, 0, st>>>(d_grids, m, k, d_hard, d_nhard, d_next, out->nbr, out->d2);
    }
    VG_HIP(hipGetLastError());
    // 3. covariances and normals
    k_cov_normals<<<grid_of(m), 256, 0, st>>>(out->xyz, out->nbr, m, k, sensor[0], sensor[1], sensor[2], out->cov,
                                               out->cov_raw, out->nrm);
    VG_HIP(hipGetLastError());
    VG_HIP(hipMemcpyAsync(out->first, out->xyz, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
    VG_HIP(hipStreamSynchronize(st));
    return VG_OK;
}

}  // namespace vg
