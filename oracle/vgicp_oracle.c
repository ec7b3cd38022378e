/*
 * FP64 CPU oracle for voxelized-GICP (VGICP) scan-matching factors.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the device library and is never on the product path.
 *
 * It is the plain definition of what one factor computes, written for
 * clarity: absolute FP64 coordinates, floor() keys, a sorted voxel list with
 * binary-search lookup, explicit 3x6 Jacobians and a Cholesky 3x3 inverse.
 *
 * Paper references (GLIM, Koide et al., 2024):
 *   Sec. III-C "Preprocessing": Gaussian voxel map, per-voxel average of the
 *       member points' means and covariances, resolutions r_0 * 2^(l-1).
 *   Sec. III-C "Correspondence search": visibility test on the surface normal
 *       and the voxel coordinate q = floor(p / r).
 *   Sec. III-C Eq. (em), Eq. (d2d): e = sum_l sum_k d^T (C~ + R C R^T)^-1 d.
 *   Sec. III-C "Linearization": Omega frozen at the linearization point,
 *       A_k = [R (mu)x, -R], H = sum A^T Omega A, b = sum A^T Omega d.
 *
 * Readings taken where the paper is loose (each one is pinned by a test):
 *   - the factor pose T maps source-frame points into the target frame,
 *     y = R mu + t, and the voxel key is floor(y / r) of the transformed point;
 *   - the covariance term is R C R^T (a pose does not translate a covariance);
 *   - H and b are 6x6 / 6-vectors w.r.t. a right perturbation T Exp(xi) with
 *     xi = [omega; v]; e carries no factor 1/2, so the Gauss-Newton step is
 *     delta = -H^-1 b;
 *   - a point with no voxel at a level contributes nothing there; levels are
 *     summed with equal weight; a point is discarded at every level when
 *     (mu - T^-1 c) . n > 0 with c the target viewpoint.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -o liboracle.so vgicp_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_NOT_SPD (-6)
#define ORC_ERR_ARG (-1)

typedef struct {
    double r;            /* voxel size of this level */
    int64_t n;           /* number of voxels */
    const int64_t *key;  /* n x 3, ascending lexicographic (x, y, z) */
    const double *mean;  /* n x 3 */
    const double *cov;   /* n x 6: xx xy xz yy yz zz */
} orc_level;

typedef struct {
    int64_t n;                 /* number of source points */
    const double *xyz;         /* n x 3 source means, source frame */
    const double *cov;         /* n x 6 source covariances, source frame */
    const double *nrm;         /* n x 3 normals (may be NULL when validate == 0) */
    int32_t L;                 /* number of levels */
    const orc_level *levels;   /* the target's voxel map, one entry per level */
    const double *viewpoint;   /* target sensor position, target frame */
    int32_t validate;          /* 1: surface-orientation correspondence validation */
    const int64_t *frozen;     /* NULL, or n x L voxel indices (-1: none) used instead of lookups */
    const double *omega_pose;  /* NULL, or a pose whose rotation defines Omega (frozen Omega) */
} orc_problem;

int32_t orc_version(void) { return 3; }

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                        */

static void sym6_to_mat(const double c[6], double M[9]) {
    M[0] = c[0]; M[1] = c[1]; M[2] = c[2];
    M[3] = c[1]; M[4] = c[3]; M[5] = c[4];
    M[6] = c[2]; M[7] = c[4]; M[8] = c[5];
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void transpose3(const double A[9], double T[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * j + i] = A[3 * i + j];
}

static void hat(const double v[3], double S[9]) {
    S[0] = 0.0;   S[1] = -v[2]; S[2] = v[1];
    S[3] = v[2];  S[4] = 0.0;   S[5] = -v[0];
    S[6] = -v[1]; S[7] = v[0];  S[8] = 0.0;
}

/* Inverse of a symmetric positive definite 3x3 matrix through M = L L^T. */
static int spd_inverse3(const double M[9], double Minv[9]) {
    double L[9] = {0};
    for (int j = 0; j < 3; ++j) {
        double s = M[3 * j + j];
        for (int k = 0; k < j; ++k) s -= L[3 * j + k] * L[3 * j + k];
        if (!(s > 0.0)) return ORC_ERR_NOT_SPD;
        L[3 * j + j] = sqrt(s);
        for (int i = j + 1; i < 3; ++i) {
            double u = M[3 * i + j];
            for (int k = 0; k < j; ++k) u -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = u / L[3 * j + j];
        }
    }
    /* X = L^-1 (lower triangular) */
    double X[9] = {0};
    for (int c = 0; c < 3; ++c) {
        for (int i = 0; i < 3; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[3 * i + k] * X[3 * k + c];
            X[3 * i + c] = s / L[3 * i + i];
        }
    }
    /* M^-1 = X^T X */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += X[3 * k + i] * X[3 * k + j];
            Minv[3 * i + j] = s;
        }
    return ORC_OK;
}

/* Solve the 6x6 SPD system A x = y by Cholesky; returns ORC_ERR_NOT_SPD if it fails. */
static int spd_solve6(const double A[36], const double y[6], double x[6]) {
    double L[36] = {0};
    for (int j = 0; j < 6; ++j) {
        double s = A[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (!(s > 0.0)) return ORC_ERR_NOT_SPD;
        L[6 * j + j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double u = A[6 * i + j];
            for (int k = 0; k < j; ++k) u -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = u / L[6 * j + j];
        }
    }
    double z[6];
    for (int i = 0; i < 6; ++i) {
        double s = y[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * z[k];
        z[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
        x[i] = s / L[6 * i + i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* voxelization (Sec. III-C, Preprocessing)                                   */

typedef struct {
    int64_t k[3];
    int64_t idx;
} keyed_point;

static int cmp_keyed(const void *a, const void *b) {
    const keyed_point *p = (const keyed_point *)a, *q = (const keyed_point *)b;
    for (int i = 0; i < 3; ++i) {
        if (p->k[i] < q->k[i]) return -1;
        if (p->k[i] > q->k[i]) return 1;
    }
    return (p->idx < q->idx) ? -1 : (p->idx > q->idx);
}

static int cmp_key3(const int64_t *a, const int64_t *b) {
    for (int i = 0; i < 3; ++i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}

/*
 * Gaussian voxel map of one level: every point falls in voxel floor(x / r);
 * a voxel stores the average of its points' means and the average of their
 * covariances.  Voxels are returned in ascending lexicographic key order (the
 * canonical voxel index is that rank); sums run in ascending point index.
 * Output arrays must hold n entries.  Returns the number of voxels.
 */
int64_t orc_voxelize(const double *xyz, const double *cov, int64_t n, double r,
                     int64_t *key_out, double *mean_out, double *cov_out, int64_t *count_out) {
    if (n <= 0) return 0;
    keyed_point *kp = (keyed_point *)malloc((size_t)n * sizeof(keyed_point));
    if (!kp) return ORC_ERR_ARG;
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) kp[i].k[a] = (int64_t)floor(xyz[3 * i + a] / r);
        kp[i].idx = i;
    }
    qsort(kp, (size_t)n, sizeof(keyed_point), cmp_keyed);
    int64_t v = -1;
    double sm[3] = {0}, sc[6] = {0};
    int64_t cnt = 0;
    for (int64_t s = 0; s <= n; ++s) {
        int boundary = (s == n) || (s == 0) || cmp_key3(kp[s].k, kp[s - 1].k) != 0;
        if (boundary && s > 0) {
            for (int a = 0; a < 3; ++a) mean_out[3 * v + a] = sm[a] / (double)cnt;
            for (int a = 0; a < 6; ++a) cov_out[6 * v + a] = sc[a] / (double)cnt;
            count_out[v] = cnt;
        }
        if (s == n) break;
        if (boundary) {
            ++v;
            for (int a = 0; a < 3; ++a) key_out[3 * v + a] = kp[s].k[a];
            memset(sm, 0, sizeof sm);
            memset(sc, 0, sizeof sc);
            cnt = 0;
        }
        int64_t i = kp[s].idx;
        for (int a = 0; a < 3; ++a) sm[a] += xyz[3 * i + a];
        for (int a = 0; a < 6; ++a) sc[a] += cov[6 * i + a];
        ++cnt;
    }
    free(kp);
    return v + 1;
}

/* Voxel index of `key` in a level, or -1. */
int64_t orc_lookup(const orc_level *lv, const int64_t key[3]) {
    int64_t lo = 0, hi = lv->n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_key3(lv->key + 3 * mid, key);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* the factor (Sec. III-C, Correspondence search + Linearization)             */

static void transform(const double pose[12], const double x[3], double y[3]) {
    for (int i = 0; i < 3; ++i)
        y[i] = pose[3 * i + 0] * x[0] + pose[3 * i + 1] * x[1] + pose[3 * i + 2] * x[2] + pose[9 + i];
}

/* Surface-orientation test: visible unless (mu - T^-1 c) . n > 0. */
static int visible(const orc_problem *p, const double pose[12], int64_t k) {
    if (!p->validate) return 1;
    const double *R = pose, *t = pose + 9, *c = p->viewpoint;
    double dc[3] = {c[0] - t[0], c[1] - t[1], c[2] - t[2]};
    double cs[3];   /* T^-1 c = R^T (c - t) */
    for (int i = 0; i < 3; ++i) cs[i] = R[0 * 3 + i] * dc[0] + R[1 * 3 + i] * dc[1] + R[2 * 3 + i] * dc[2];
    const double *mu = p->xyz + 3 * k, *n = p->nrm + 3 * k;
    double s = (mu[0] - cs[0]) * n[0] + (mu[1] - cs[1]) * n[1] + (mu[2] - cs[2]) * n[2];
    return !(s > 0.0);
}

/*
 * Terms of one (point, voxel) pair: e += d^T W d, H += J^T W J, b += J^T W d with
 * d = mu~ - (R mu + t), W = (C~ + Rw C Rw^T)^-1 (Rw = R unless Omega is frozen)
 * and J = dd/dxi = [R (mu)x, -R].
 */
static int pair_terms(const double pose[12], const double Rw[9], const double mu[3], const double c6[6],
                      const double vmean[3], const double vcov[6], double *e, double H[36], double b[6]) {
    const double *R = pose;
    double y[3], d[3];
    transform(pose, mu, y);
    for (int i = 0; i < 3; ++i) d[i] = vmean[i] - y[i];
    double C[9], Cv[9], RC[9], RwT[9], RCRt[9], M[9], W[9];
    sym6_to_mat(c6, C);
    sym6_to_mat(vcov, Cv);
    matmul3(Rw, C, RC);
    transpose3(Rw, RwT);
    matmul3(RC, RwT, RCRt);
    for (int i = 0; i < 9; ++i) M[i] = Cv[i] + RCRt[i];
    /* symmetrize against rounding in the product */
    M[1] = M[3] = 0.5 * (M[1] + M[3]);
    M[2] = M[6] = 0.5 * (M[2] + M[6]);
    M[5] = M[7] = 0.5 * (M[5] + M[7]);
    int st = spd_inverse3(M, W);
    if (st != ORC_OK) return st;
    double S[9], RS[9], J[18];
    hat(mu, S);
    matmul3(R, S, RS);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            J[6 * i + j] = RS[3 * i + j];
            J[6 * i + 3 + j] = -R[3 * i + j];
        }
    double WJ[18], Wd[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += W[3 * i + k] * J[6 * k + j];
            WJ[6 * i + j] = s;
        }
        Wd[i] = W[3 * i + 0] * d[0] + W[3 * i + 1] * d[1] + W[3 * i + 2] * d[2];
    }
    *e += d[0] * Wd[0] + d[1] * Wd[1] + d[2] * Wd[2];
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += J[6 * k + i] * WJ[6 * k + j];
            H[6 * i + j] += s;
        }
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += J[6 * k + i] * Wd[k];
        b[i] += s;
    }
    return ORC_OK;
}

/*
 * Linearize one factor at `pose`.  Outputs: e, H (6x6 row-major), b (6),
 * inliers per level.  Optional per (point, level) traces (NULL to skip):
 * keys n*L*3, voxel index n*L (-1: none or discarded), distance of y to the
 * nearest face of its voxel n*L, visibility n.
 */
int orc_linearize(const orc_problem *p, const double pose[12], double *e, double H[36], double b[6],
                  int64_t *inliers, int64_t *tr_key, int64_t *tr_vidx, double *tr_face, int32_t *tr_vis) {
    *e = 0.0;
    memset(H, 0, 36 * sizeof(double));
    memset(b, 0, 6 * sizeof(double));
    for (int l = 0; l < p->L; ++l) inliers[l] = 0;
    const double *Rw = p->omega_pose ? p->omega_pose : pose;
    for (int64_t k = 0; k < p->n; ++k) {
        const double *mu = p->xyz + 3 * k;
        int vis = p->frozen ? 1 : visible(p, pose, k);
        if (tr_vis) tr_vis[k] = vis;
        double y[3];
        transform(pose, mu, y);
        for (int l = 0; l < p->L; ++l) {
            const orc_level *lv = &p->levels[l];
            int64_t q[3];
            for (int a = 0; a < 3; ++a) q[a] = (int64_t)floor(y[a] / lv->r);
            int64_t v;
            if (p->frozen) v = p->frozen[k * p->L + l];
            else v = vis ? orc_lookup(lv, q) : -1;
            if (tr_key) for (int a = 0; a < 3; ++a) tr_key[(k * p->L + l) * 3 + a] = q[a];
            if (tr_vidx) tr_vidx[k * p->L + l] = v;
            if (tr_face) {
                double m = INFINITY;
                for (int a = 0; a < 3; ++a) {
                    double lo = y[a] - (double)q[a] * lv->r, hi = (double)(q[a] + 1) * lv->r - y[a];
                    if (lo < m) m = lo;
                    if (hi < m) m = hi;
                }
                tr_face[k * p->L + l] = m;
            }
            if (v < 0) continue;
            int st = pair_terms(pose, Rw, mu, p->cov + 6 * k, lv->mean + 3 * v, lv->cov + 6 * v, e, H, b);
            if (st != ORC_OK) return st;
            inliers[l] += 1;
        }
    }
    return ORC_OK;
}

/*
 * Terms (e, H, b packed as 1 + 36 + 6 doubles) of point k at level l when it is
 * matched to the voxel with key `key`.  Returns 1 if that voxel exists, 0 if not
 * (out is then zero), or an error code.  Used to account for points lying so
 * close to a voxel face that either neighbouring key is a correct answer.
 */
int orc_point_terms(const orc_problem *p, const double pose[12], int64_t k, int32_t l,
                    const int64_t key[3], double out[43]) {
    memset(out, 0, 43 * sizeof(double));
    const orc_level *lv = &p->levels[l];
    int64_t v = orc_lookup(lv, key);
    if (v < 0) return 0;
    const double *Rw = p->omega_pose ? p->omega_pose : pose;
    int st = pair_terms(pose, Rw, p->xyz + 3 * k, p->cov + 6 * k, lv->mean + 3 * v, lv->cov + 6 * v,
                        out, out + 1, out + 37);
    return st == ORC_OK ? 1 : st;
}

/*
 * Scale of the gradient's summands: over every matched (point, level) pair,
 * the sum of the Euclidean norms of its contribution to the rotation half
 * b[0..2] and to the translation half b[3..5] of b.  Near convergence the
 * contributions cancel, so |b| is far below this sum; errors of a device sum
 * are then stated against this scale.  out[0]: rotation half, out[1]:
 * translation half.
 */
int orc_gradient_scale(const orc_problem *p, const double pose[12], double out[2]) {
    out[0] = 0.0;
    out[1] = 0.0;
    const double *Rw = p->omega_pose ? p->omega_pose : pose;
    for (int64_t k = 0; k < p->n; ++k) {
        const double *mu = p->xyz + 3 * k;
        int vis = p->frozen ? 1 : visible(p, pose, k);
        double y[3];
        transform(pose, mu, y);
        for (int l = 0; l < p->L; ++l) {
            const orc_level *lv = &p->levels[l];
            int64_t q[3];
            for (int a = 0; a < 3; ++a) q[a] = (int64_t)floor(y[a] / lv->r);
            int64_t v;
            if (p->frozen) v = p->frozen[k * p->L + l];
            else v = vis ? orc_lookup(lv, q) : -1;
            if (v < 0) continue;
            double e1 = 0.0, H1[36] = {0}, b1[6] = {0};
            int st = pair_terms(pose, Rw, mu, p->cov + 6 * k, lv->mean + 3 * v, lv->cov + 6 * v, &e1, H1, b1);
            if (st != ORC_OK) return st;
            out[0] += sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
            out[1] += sqrt(b1[3] * b1[3] + b1[4] * b1[4] + b1[5] * b1[5]);
        }
    }
    return ORC_OK;
}

/* e at `pose` (correspondences and Omega recomputed there unless frozen). */
int orc_evaluate(const orc_problem *p, const double pose[12], double *e) {
    double H[36], b[6];
    int64_t inl[64];
    if (p->L > 64) return ORC_ERR_ARG;
    return orc_linearize(p, pose, e, H, b, inl, NULL, NULL, NULL, NULL);
}

/*
 * Exact gradient of e(T Exp(xi)) at xi = 0, with Omega = (C~ + R C R^T)^-1
 * recomputed (not frozen) and the correspondences found at `pose` held fixed:
 *   de/dxi_j = 2 (J e_j)^T W d - (W d)^T (dM/dxi_j) (W d),
 *   dM/domega_j = R (hat(e_j) C - C hat(e_j)) R^T,  dM/dv_j = 0,
 *   de/dmu_k = -2 R^T W d   (summed over levels).
 * g_mu may be NULL.
 */
int orc_gradient(const orc_problem *p, const double pose[12], double g_xi[6], double *g_mu) {
    const double *R = pose;
    memset(g_xi, 0, 6 * sizeof(double));
    if (g_mu) memset(g_mu, 0, (size_t)p->n * 3 * sizeof(double));
    double Rt[9];
    transpose3(R, Rt);
    for (int64_t k = 0; k < p->n; ++k) {
        const double *mu = p->xyz + 3 * k;
        int vis = p->frozen ? 1 : visible(p, pose, k);
        double y[3];
        transform(pose, mu, y);
        for (int l = 0; l < p->L; ++l) {
            const orc_level *lv = &p->levels[l];
            int64_t v;
            if (p->frozen) v = p->frozen[k * p->L + l];
            else {
                int64_t q[3];
                for (int a = 0; a < 3; ++a) q[a] = (int64_t)floor(y[a] / lv->r);
                v = vis ? orc_lookup(lv, q) : -1;
            }
            if (v < 0) continue;
            double d[3];
            for (int i = 0; i < 3; ++i) d[i] = lv->mean[3 * v + i] - y[i];
            double C[9], Cv[9], RC[9], RCRt[9], M[9], W[9];
            sym6_to_mat(p->cov + 6 * k, C);
            sym6_to_mat(lv->cov + 6 * v, Cv);
            matmul3(R, C, RC);
            matmul3(RC, Rt, RCRt);
            for (int i = 0; i < 9; ++i) M[i] = Cv[i] + RCRt[i];
            M[1] = M[3] = 0.5 * (M[1] + M[3]);
            M[2] = M[6] = 0.5 * (M[2] + M[6]);
            M[5] = M[7] = 0.5 * (M[5] + M[7]);
            int st = spd_inverse3(M, W);
            if (st != ORC_OK) return st;
            double u[3];   /* W d */
            for (int i = 0; i < 3; ++i) u[i] = W[3 * i] * d[0] + W[3 * i + 1] * d[1] + W[3 * i + 2] * d[2];
            /* J = [R hat(mu), -R] */
            double S[9], RS[9];
            hat(mu, S);
            matmul3(R, S, RS);
            for (int j = 0; j < 3; ++j) {
                double jw = RS[0 * 3 + j] * u[0] + RS[1 * 3 + j] * u[1] + RS[2 * 3 + j] * u[2];
                double jv = -(R[0 * 3 + j] * u[0] + R[1 * 3 + j] * u[1] + R[2 * 3 + j] * u[2]);
                /* dM/domega_j */
                double E[9], EC[9], CE[9], Dm[9], tmp[9], dM[9];
                double ej[3] = {0, 0, 0};
                ej[j] = 1.0;
                hat(ej, E);
                matmul3(E, C, EC);
                matmul3(C, E, CE);
                for (int i = 0; i < 9; ++i) Dm[i] = EC[i] - CE[i];
                matmul3(R, Dm, tmp);
                matmul3(tmp, Rt, dM);
                double q = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) q += u[a] * dM[3 * a + c] * u[c];
                g_xi[j] += 2.0 * jw - q;
                g_xi[3 + j] += 2.0 * jv;
            }
            if (g_mu) {
                for (int i = 0; i < 3; ++i)
                    g_mu[3 * k + i] += -2.0 * (Rt[3 * i] * u[0] + Rt[3 * i + 1] * u[1] + Rt[3 * i + 2] * u[2]);
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SE(3) exponential and a Levenberg-Marquardt driver                         */

/* Exp of xi = [omega; v]: R = Rodrigues(omega), t = V v with
 * V = I + (1 - cos th)/th^2 W + (th - sin th)/th^3 W^2, W = hat(omega). */
void orc_se3_exp(const double xi[6], double out[12]) {
    const double *w = xi, *v = xi + 3;
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double A, B, Cc;  /* sin th/th, (1-cos th)/th^2, (th - sin th)/th^3 */
    if (th < 1e-5) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        Cc = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        Cc = (th - sin(th)) / (th2 * th);
    }
    double W[9], W2[9];
    hat(w, W);
    matmul3(W, W, W2);
    double Rm[9], V[9];
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        Rm[i] = I + A * W[i] + B * W2[i];
        V[i] = I + B * W[i] + Cc * W2[i];
    }
    for (int i = 0; i < 9; ++i) out[i] = Rm[i];
    for (int i = 0; i < 3; ++i) out[9 + i] = V[3 * i] * v[0] + V[3 * i + 1] * v[1] + V[3 * i + 2] * v[2];
}

/* a * b for poses stored as 12 doubles. */
void orc_pose_mul(const double a[12], const double b[12], double out[12]) {
    double Rm[9];
    matmul3(a, b, Rm);
    double t[3];
    for (int i = 0; i < 3; ++i)
        t[i] = a[3 * i] * b[9] + a[3 * i + 1] * b[10] + a[3 * i + 2] * b[11] + a[9 + i];
    memcpy(out, Rm, sizeof Rm);
    memcpy(out + 9, t, sizeof t);
}

/*
 * Levenberg-Marquardt on one factor: at each iteration linearize at T, solve
 * (H + lambda diag(H)) delta = -b, propose T Exp(delta), accept it when its
 * error is lower (lambda /= 10) and otherwise keep T (lambda *= 10).
 * Outputs the final pose, the accept flags and e at each linearization.
 */
int orc_lm(const orc_problem *p, const double pose_in[12], int32_t iters, double lambda0,
           double pose_out[12], int32_t *accepted, double *e_hist, double *lambda_out) {
    double T[12];
    memcpy(T, pose_in, sizeof T);
    double lambda = lambda0;
    int64_t inl[64];
    if (p->L > 64) return ORC_ERR_ARG;
    for (int it = 0; it < iters; ++it) {
        double e, H[36], b[6];
        int st = orc_linearize(p, T, &e, H, b, inl, NULL, NULL, NULL, NULL);
        if (st != ORC_OK) return st;
        if (e_hist) e_hist[it] = e;
        double A[36], rhs[6], delta[6];
        memcpy(A, H, sizeof A);
        for (int i = 0; i < 6; ++i) {
            A[6 * i + i] += lambda * H[6 * i + i];
            rhs[i] = -b[i];
        }
        int ok = spd_solve6(A, rhs, delta) == ORC_OK;
        int acc = 0;
        if (ok) {
            double E[12], Tn[12], en;
            orc_se3_exp(delta, E);
            orc_pose_mul(T, E, Tn);
            st = orc_evaluate(p, Tn, &en);
            if (st != ORC_OK) return st;
            if (en < e) {
                memcpy(T, Tn, sizeof T);
                acc = 1;
            }
        }
        if (acc) lambda /= 10.0; else lambda *= 10.0;
        if (accepted) accepted[it] = acc;
    }
    memcpy(pose_out, T, sizeof T);
    if (lambda_out) *lambda_out = lambda;
    return ORC_OK;
}
