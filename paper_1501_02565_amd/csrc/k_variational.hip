// k_variational.hip -- one-level variational refinement of the interpolated
// field (Sec. 4 of the paper): an energy of a data term (colour and
// gradient constancy with a normalisation, the paper citing its form) and a
// smoothness term on the flow gradient norm weighted by alpha(x) =
// exp(-kappa ||grad I1||), minimised from the interpolated field u0 without
// coarse-to-fine by `fixed_point` steps (the non-linear weights of the
// Euler-Lagrange equations re-evaluated) of `sor` successive
// over-relaxation sweeps.
//
// The discrete problem (the reading this library takes of the cited data
// term, and its discretisation):
//   I2w = I2(x + u0(x)) bilinear, coordinates clamped; central differences
//   with the border pixel repeated; Ixx, Iyy, Ixy of I2w; Iz = I2w - I1;
//   Ixz, Iyz the gradient differences of I2w and I1;
//   colour   sum_c theta_c (Iz + Ix du + Iy dv)^2,      theta_c  = 1/(Ix^2+Iy^2+zeta^2)
//   gradient sum_c thetax_c (Ixz + Ixx du + Ixy dv)^2 + thetay_c (Iyz + Ixy du + Iyy dv)^2,
//            thetax = 1/(Ixx^2+Ixy^2+zeta^2), thetay = 1/(Ixy^2+Iyy^2+zeta^2)
//   E = sum_x delta psi(colour) + gamma psi(gradient)
//     + sum over 4-neighbour edges lam (alpha_i+alpha_j)/2 psi(|U_j-U_i|^2 + |V_j-V_i|^2)
//   psi(s^2) = sqrt(s^2 + eps^2), U = u0 + du, V = v0 + dv.
// Each fixed-point step evaluates psi' at the current (du, dv) and solves
//   (A11 + sum_j g_ij) du_i + A12 dv_i = b1 + sum_j g_ij (U_j - u0_i), likewise dv,
// by red-black SOR sweeps (red: x + y even), du before dv at each pixel; an
// equation with a zero diagonal leaves its unknown unchanged.
//
// Kernels (all pixel-parallel, FP32, one rounding per operation where it
// matters; streaming and bound by HBM):
//   k_var_warp     I2w
//   k_var_coef     per pixel the colour and gradient systems J (6 entries
//                  each) and alpha, stored as 13 planes
//   k_var_weights  per pixel A11 A12 A22 b1 b2, per edge g (right, down)
//   k_var_sor      one colour of one sweep (a pixel's 4 neighbours all have
//                  the other colour, so a launch updates without races)
//   k_var_out      u0 + du
#include "epic_dev.h"

namespace epic {

namespace {

__device__ __forceinline__ float psi_d(float s2, float eps) {
    return 0.5f / sqrtf(fmaxf(s2, 0.0f) + eps * eps);
}

__device__ __forceinline__ float quad(const float* J, float du, float dv) {
    return J[0] * du * du + 2.0f * J[1] * du * dv + J[2] * dv * dv + 2.0f * J[3] * du + 2.0f * J[4] * dv + J[5];
}

}  // namespace

__global__ __launch_bounds__(256) void k_var_warp(VarArgs A) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    const int W = A.W, H = A.H, C = A.C;
    const int x = (int)(i % W), y = (int)(i / W);
    const float fxp = fminf(fmaxf((float)x + A.u0[2 * i], 0.0f), (float)(W - 1));
    const float fyp = fminf(fmaxf((float)y + A.u0[2 * i + 1], 0.0f), (float)(H - 1));
    const int x0 = min((int)floorf(fxp), W > 1 ? W - 2 : 0), y0 = min((int)floorf(fyp), H > 1 ? H - 2 : 0);
    const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
    const float fx = fxp - (float)x0, fy = fyp - (float)y0;
    for (int c = 0; c < C; ++c) {
        const float a = A.I2[((long long)y0 * W + x0) * C + c], b = A.I2[((long long)y0 * W + x1) * C + c];
        const float d = A.I2[((long long)y1 * W + x0) * C + c], e = A.I2[((long long)y1 * W + x1) * C + c];
        A.I2w[i * C + c] = (1.0f - fy) * ((1.0f - fx) * a + fx * b) + fy * ((1.0f - fx) * d + fx * e);
    }
}

__global__ __launch_bounds__(256) void k_var_coef(VarArgs A) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    const int W = A.W, H = A.H, C = A.C;
    const int x = (int)(i % W), y = (int)(i / W);
    const int xl = max(x - 1, 0), xr = min(x + 1, W - 1), yu = max(y - 1, 0), yd = min(y + 1, H - 1);
    auto at = [&](const float* img, int yy, int xx, int c) { return img[((long long)yy * W + xx) * C + c]; };
    float J[12];
    for (int k = 0; k < 12; ++k) J[k] = 0.0f;
    float gn = 0.0f;
    const float z2 = A.zeta * A.zeta;
    for (int c = 0; c < C; ++c) {
        const float w = at(A.I2w, y, x, c);
        const float Ix = 0.5f * (at(A.I2w, y, xr, c) - at(A.I2w, y, xl, c));
        const float Iy = 0.5f * (at(A.I2w, yd, x, c) - at(A.I2w, yu, x, c));
        const float gx1 = 0.5f * (at(A.I1, y, xr, c) - at(A.I1, y, xl, c));
        const float gy1 = 0.5f * (at(A.I1, yd, x, c) - at(A.I1, yu, x, c));
        const float Iz = w - at(A.I1, y, x, c);
        const float Ixx = at(A.I2w, y, xr, c) - 2.0f * w + at(A.I2w, y, xl, c);
        const float Iyy = at(A.I2w, yd, x, c) - 2.0f * w + at(A.I2w, yu, x, c);
        const float Ixy = 0.25f * (at(A.I2w, yd, xr, c) - at(A.I2w, yd, xl, c) - at(A.I2w, yu, xr, c) +
                                   at(A.I2w, yu, xl, c));
        const float Ixz = Ix - gx1, Iyz = Iy - gy1;
        const float th = 1.0f / (Ix * Ix + Iy * Iy + z2);
        const float thx = 1.0f / (Ixx * Ixx + Ixy * Ixy + z2);
        const float thy = 1.0f / (Ixy * Ixy + Iyy * Iyy + z2);
        // colour system: th [Ix Iy Iz]^T [Ix Iy Iz]
        J[0] += th * Ix * Ix; J[1] += th * Ix * Iy; J[2] += th * Iy * Iy;
        J[3] += th * Ix * Iz; J[4] += th * Iy * Iz; J[5] += th * Iz * Iz;
        // gradient system: thx [Ixx Ixy Ixz]^T [..] + thy [Ixy Iyy Iyz]^T [..]
        J[6] += thx * Ixx * Ixx + thy * Ixy * Ixy;
        J[7] += thx * Ixx * Ixy + thy * Ixy * Iyy;
        J[8] += thx * Ixy * Ixy + thy * Iyy * Iyy;
        J[9] += thx * Ixx * Ixz + thy * Ixy * Iyz;
        J[10] += thx * Ixy * Ixz + thy * Iyy * Iyz;
        J[11] += thx * Ixz * Ixz + thy * Iyz * Iyz;
        gn += gx1 * gx1 + gy1 * gy1;
    }
    for (int k = 0; k < 12; ++k) A.coef[(long long)k * A.HW + i] = J[k];
    A.coef[12LL * A.HW + i] = expf(-A.kappa * sqrtf(gn));
}

__global__ __launch_bounds__(256) void k_var_weights(VarArgs A) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    const int W = A.W, H = A.H;
    const int x = (int)(i % W), y = (int)(i / W);
    float JC[6], JG[6];
    for (int k = 0; k < 6; ++k) {
        JC[k] = A.coef[(long long)k * A.HW + i];
        JG[k] = A.coef[(long long)(6 + k) * A.HW + i];
    }
    const float du = A.du[i], dv = A.dv[i];
    const float wc = A.delta * psi_d(quad(JC, du, dv), A.eps);
    const float wg = A.gamma * psi_d(quad(JG, du, dv), A.eps);
    A.sys[i] = wc * JC[0] + wg * JG[0];
    A.sys[A.HW + i] = wc * JC[1] + wg * JG[1];
    A.sys[2 * A.HW + i] = wc * JC[2] + wg * JG[2];
    A.sys[3 * A.HW + i] = -(wc * JC[3] + wg * JG[3]);
    A.sys[4 * A.HW + i] = -(wc * JC[4] + wg * JG[4]);
    const float* alpha = A.coef + 12LL * A.HW;
    const float U = A.u0[2 * i] + du, V = A.u0[2 * i + 1] + dv;
    // edge to the right and edge down (0 where there is none)
    float gx = 0.0f, gy = 0.0f;
    if (x + 1 < W) {
        const long long j = i + 1;
        const float dU = (A.u0[2 * j] + A.du[j]) - U, dV = (A.u0[2 * j + 1] + A.dv[j]) - V;
        gx = A.lam * 0.5f * (alpha[i] + alpha[j]) * psi_d(dU * dU + dV * dV, A.eps);
    }
    if (y + 1 < H) {
        const long long j = i + W;
        const float dU = (A.u0[2 * j] + A.du[j]) - U, dV = (A.u0[2 * j + 1] + A.dv[j]) - V;
        gy = A.lam * 0.5f * (alpha[i] + alpha[j]) * psi_d(dU * dU + dV * dV, A.eps);
    }
    A.sys[5 * A.HW + i] = gx;
    A.sys[6 * A.HW + i] = gy;
}

// one thread per pixel of the colour: row y holds ceil(W / 2) slots, slot k
// the pixel x = 2k + ((y + color) & 1) when that lies inside the row
__global__ __launch_bounds__(256) void k_var_sor(VarArgs A, int color) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const int W = A.W, H = A.H;
    const int Wh = (W + 1) >> 1;
    if (t >= (long long)Wh * H) return;
    const int y = (int)(t / Wh);
    const int x = 2 * (int)(t % Wh) + ((y + color) & 1);
    if (x >= W) return;
    const long long i = (long long)y * W + x;
    const float* gxa = A.sys + 5LL * A.HW;
    const float* gya = A.sys + 6LL * A.HW;
    const float u0i = A.u0[2 * i], v0i = A.u0[2 * i + 1];
    float sw = 0.0f, su = 0.0f, sv = 0.0f;
    auto nb = [&](long long j, float g) {
        sw += g;
        su += g * ((A.u0[2 * j] + A.du[j]) - u0i);
        sv += g * ((A.u0[2 * j + 1] + A.dv[j]) - v0i);
    };
    if (x + 1 < W) nb(i + 1, gxa[i]);
    if (x > 0) nb(i - 1, gxa[i - 1]);
    if (y + 1 < H) nb(i + W, gya[i]);
    if (y > 0) nb(i - W, gya[i - W]);
    const float a11 = A.sys[i], a12 = A.sys[A.HW + i], a22 = A.sys[2 * A.HW + i];
    const float b1 = A.sys[3 * A.HW + i], b2 = A.sys[4 * A.HW + i];
    const float om = A.omega;
    // a zero diagonal (no image gradient, no neighbour weight) leaves the
    // equation empty: the unknown keeps its value
    const float du0 = A.du[i], dv0 = A.dv[i];
    const float du = a11 + sw > 0.0f ? (1.0f - om) * du0 + om * (b1 - a12 * dv0 + su) / (a11 + sw) : du0;
    const float dv = a22 + sw > 0.0f ? (1.0f - om) * dv0 + om * (b2 - a12 * du + sv) / (a22 + sw) : dv0;
    A.du[i] = du;
    A.dv[i] = dv;
}

__global__ __launch_bounds__(256) void k_var_out(VarArgs A) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    A.flow[2 * i] = A.u0[2 * i] + A.du[i];
    A.flow[2 * i + 1] = A.u0[2 * i + 1] + A.dv[i];
}

__global__ __launch_bounds__(256) void k_var_zero(VarArgs A) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    A.du[i] = 0.0f;
    A.dv[i] = 0.0f;
}

hipError_t launch_variational(const VarArgs& A, hipStream_t s) {
    const dim3 g((unsigned)((A.HW + 255) / 256)), b(256);
    const dim3 gs((unsigned)(((long long)((A.W + 1) >> 1) * A.H + 255) / 256));
    hipLaunchKernelGGL(k_var_zero, g, b, 0, s, A);
    hipLaunchKernelGGL(k_var_warp, g, b, 0, s, A);
    hipLaunchKernelGGL(k_var_coef, g, b, 0, s, A);
    for (int f = 0; f < A.fixed_point; ++f) {
        hipLaunchKernelGGL(k_var_weights, g, b, 0, s, A);
        for (int k = 0; k < A.sor; ++k) {
            hipLaunchKernelGGL(k_var_sor, gs, b, 0, s, A, 0);
            hipLaunchKernelGGL(k_var_sor, gs, b, 0, s, A, 1);
        }
    }
    hipLaunchKernelGGL(k_var_out, g, b, 0, s, A);
    return hipGetLastError();
}

}  // namespace epic
