// FP64 pose kernels: SE(3) retraction with its right Jacobian, and the
// Levenberg-Marquardt propose / accept steps on the device (one thread per
// factor; 6x6 systems are tiny, so the point is to stay on the device and
// avoid host round trips inside the loop).
#include "vg_device.h"

namespace vg {

__device__ __forceinline__ void hat3(const double v[3], double S[9]) {
    S[0] = 0.0;
    S[1] = -v[2];
    S[2] = v[1];
    S[3] = v[2];
    S[4] = 0.0;
    S[5] = -v[0];
    S[6] = -v[1];
    S[7] = v[0];
    S[8] = 0.0;
}

__device__ __forceinline__ void mm3(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// Exp of xi = [omega; v] in SE(3): rotation by Rodrigues' formula, translation
// V v with V = I + (1 - cos th)/th^2 W + (th - sin th)/th^3 W^2, W = (omega)x.
__device__ void se3_exp(const double xi[6], double out[12]) {
    const double th2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    const double th = sqrt(th2);
    double a, b, c;
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        b = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        c = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        const double s = sin(th), co = cos(th);
        a = s / th;
        b = (1.0 - co) / th2;
        c = (th - s) / (th2 * th);
    }
    double W[9], W2[9];
    hat3(xi, W);
    mm3(W, W, W2);
    double V[9];
    for (int k = 0; k < 9; ++k) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        out[k] = I + a * W[k] + b * W2[k];
        V[k] = I + b * W[k] + c * W2[k];
    }
    for (int i = 0; i < 3; ++i) out[9 + i] = V[3 * i] * xi[3] + V[3 * i + 1] * xi[4] + V[3 * i + 2] * xi[5];
}

__device__ void pose_mul(const double A[12], const double B[12], double C[12]) {
    double Rm[9];
    mm3(A, B, Rm);
    for (int i = 0; i < 3; ++i)
        C[9 + i] = A[3 * i] * B[9] + A[3 * i + 1] * B[10] + A[3 * i + 2] * B[11] + A[9 + i];
    for (int k = 0; k < 9; ++k) C[k] = Rm[k];
}

// Right Jacobian of SE(3): J_r(xi) = sum_n (-ad_xi)^n / (n+1)!, with
// ad_xi = [[(omega)x, 0], [(v)x, (omega)x]] for xi = [omega; v].  The series is
// summed until the term is negligible (it converges for every xi).
__device__ void se3_right_jacobian(const double xi[6], double J[36]) {
    double Wx[9], Vx[9];
    hat3(xi, Wx);
    hat3(xi + 3, Vx);
    double ad[36] = {0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            ad[6 * i + j] = -Wx[3 * i + j];
            ad[6 * (3 + i) + j] = -Vx[3 * i + j];
            ad[6 * (3 + i) + 3 + j] = -Wx[3 * i + j];
        }
    double term[36], next[36];
    for (int k = 0; k < 36; ++k) {
        term[k] = (k % 7 == 0) ? 1.0 : 0.0;
        J[k] = term[k];
    }
    for (int n = 1; n < 60; ++n) {
        double mx = 0.0;
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double s = 0.0;
                for (int q = 0; q < 6; ++q) s += term[6 * i + q] * ad[6 * q + j];
                next[6 * i + j] = s / (double)(n + 1);
            }
        for (int k = 0; k < 36; ++k) {
            term[k] = next[k];
            J[k] += term[k];
            mx = fmax(mx, fabs(term[k]));
        }
        if (mx < 1e-18) break;
    }
}

__global__ void k_se3_retract(int64_t F, const double* __restrict__ T0, const double* __restrict__ xi,
                              double* __restrict__ T, double* __restrict__ jr) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double x[6], E[12], A[12], C[12];
    for (int k = 0; k < 6; ++k) x[k] = xi[6 * f + k];
    for (int k = 0; k < 12; ++k) A[k] = T0[12 * f + k];
    se3_exp(x, E);
    pose_mul(A, E, C);
    for (int k = 0; k < 12; ++k) T[12 * f + k] = C[k];
    if (jr != nullptr) {
        double J[36];
        se3_right_jacobian(x, J);
        for (int k = 0; k < 36; ++k) jr[36 * f + k] = J[k];
    }
}

// Solve (H + lambda diag(H)) delta = -b by Cholesky; returns false if not SPD.
__device__ bool lm_solve(const double* row, double lambda, double delta[6]) {
    double A[36], L[36] = {0};
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) A[6 * i + j] = row[1 + 6 * i + j] + (i == j ? lambda * row[1 + 7 * i] : 0.0);
    for (int j = 0; j < 6; ++j) {
        double s = A[7 * j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (!(s > 0.0)) return false;
        L[7 * j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double u = A[6 * i + j];
            for (int k = 0; k < j; ++k) u -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = u / L[7 * j];
        }
    }
    double z[6];
    for (int i = 0; i < 6; ++i) {
        double s = -row[37 + i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * z[k];
        z[i] = s / L[7 * i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * delta[k];
        delta[i] = s / L[7 * i];
    }
    return true;
}

// Proposal of one damped step per factor: delta from (H + lambda diag H) delta = -b
// (FP64 Cholesky) at the linearization rows, candidate T Exp(delta).  A matrix
// that is not SPD leaves the candidate at T and marks it invalid.
__global__ void k_lm_propose(int64_t F, const double* __restrict__ out, const double* __restrict__ lambda,
                             const double* __restrict__ poses, double* __restrict__ cand, int32_t* __restrict__ valid) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* row = out + (int64_t)kOutRow * f;
    double delta[6], T[12], E[12], C[12];
    for (int k = 0; k < 12; ++k) T[k] = poses[12 * f + k];
    const bool ok = lm_solve(row, lambda[f], delta);
    if (ok) {
        se3_exp(delta, E);
        pose_mul(T, E, C);
    } else {
        for (int k = 0; k < 12; ++k) C[k] = T[k];
    }
    for (int k = 0; k < 12; ++k) cand[12 * f + k] = C[k];
    valid[f] = ok ? 1 : 0;
}

// Accept the candidate iff it is valid and its error is below the error at T
// (then lambda / 10), else keep T (lambda x 10).  Records e at T and the decision.
__global__ void k_lm_accept(int64_t F, const double* __restrict__ out, const double* __restrict__ e_new,
                            double* __restrict__ lambda, double* __restrict__ poses, const double* __restrict__ cand,
                            const int32_t* __restrict__ valid, double* __restrict__ e_out,
                            int32_t* __restrict__ accepted, int32_t stride, int32_t col) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double e0 = out[(int64_t)kOutRow * f];
    const bool acc = (valid[f] != 0) && (e_new[f] < e0);
    if (acc) {
        for (int k = 0; k < 12; ++k) poses[12 * f + k] = cand[12 * f + k];
        lambda[f] /= 10.0;
    } else {
        lambda[f] *= 10.0;
    }
    if (accepted != nullptr) accepted[(int64_t)stride * f + col] = acc ? 1 : 0;
    if (e_out != nullptr) e_out[(int64_t)stride * f + col] = e0;
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

vg_status launch_se3_retract(vg_context* ctx, int64_t F, const double* d_T0, const double* d_xi, double* d_T,
                             double* d_jr) {
    if (F == 0) return VG_OK;
    k_se3_retract<<<(int)((F + 63) / 64), 64, 0, ctx->stream>>>(F, d_T0, d_xi, d_T, d_jr);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

vg_status launch_lm_propose(vg_batch* b, const double* d_out, const double* d_lambda, const double* d_poses,
                            double* d_cand, int32_t* d_valid) {
    k_lm_propose<<<(int)((b->F + 63) / 64), 64, 0, b->ctx->stream>>>(b->F, d_out, d_lambda, d_poses, d_cand,
                                                                     d_valid);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

vg_status launch_lm_accept(vg_batch* b, const double* d_out, const double* d_e_new, double* d_lambda,
                           double* d_poses, const double* d_cand, const int32_t* d_valid, double* d_e,
                           int32_t* d_accepted, int32_t stride, int32_t col) {
    k_lm_accept<<<(int)((b->F + 63) / 64), 64, 0, b->ctx->stream>>>(b->F, d_out, d_e_new, d_lambda, d_poses, d_cand,
                                                                    d_valid, d_e, d_accepted, stride, col);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

vg_status launch_fill(vg_context* ctx, double* d_ptr, int64_t n, double v) {
    if (n <= 0) return VG_OK;
    k_fill<<<(int)((n + 255) / 256), 256, 0, ctx->stream>>>(d_ptr, n, v);
    VG_HIP(hipGetLastError());
    return VG_OK;
}

}  // namespace vg
