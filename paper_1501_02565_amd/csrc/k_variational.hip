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
// equation with a zero diagonal leaves its unknown unchanged.  The sums are
// taken as sum_j g_ij (u0_j - u0_i) + sum_j g_ij du_j: the first part is
// fixed for a fixed-point step and folded into the right-hand side, and the
// small increments du carry the sweeps (no cancellation against u0).
//
// Kernels (FP32):
//   k_var_warp     I2w (pixel-parallel)
//   k_var_coef     per pixel the colour and gradient systems J (6 entries
//                  each) and alpha, stored as 13 planes
//   k_var_weights  per fixed-point step and pixel the 9 numbers its update
//                  needs: omega / D1 and omega / D2 for the diagonals
//                  D1 = A11 + sum g, D2 = A22 + sum g (one division per
//                  step, not per sweep), A12, right-hand sides B1, B2, and
//                  its 4 edge weights
//                  (each edge evaluated in one canonical order, so both
//                  endpoints hold the same value)
//   k_var_sor      S half-sweeps per launch with the sweeps blocked in time:
//                  a workgroup loads its tile and a halo of S pixels into
//                  LDS (du, dv, the two colours in separate arrays) and its
//                  pixels' 9 numbers into registers, relaxes the whole
//                  region S times (each half-sweep corrupts at most one
//                  more ring from the region's edge inwards, so the tile's
//                  values equal those of S global half-sweeps) and writes
//                  the tile to the other buffer of a ping-pong pair.  A
//                  launch per half-sweep would spend most of its time in
//                  launching and in re-reading the system from memory.
//   k_var_out      u0 + du
#include <type_traits>

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

// Edge (p, q) with p the left or upper pixel: lam (alpha_p + alpha_q) / 2
// psi'(|U_q - U_p|^2 + |V_q - V_p|^2), in this one order for both ends.
__device__ __forceinline__ float edge_weight(const VarArgs& A, const float* du, const float* dv, long long p,
                                             long long q) {
    const float* alpha = A.coef + 12LL * A.HW;
    const float dU = (A.u0[2 * q] + du[q]) - (A.u0[2 * p] + du[p]);
    const float dV = (A.u0[2 * q + 1] + dv[q]) - (A.u0[2 * p + 1] + dv[p]);
    return A.lam * 0.5f * (alpha[p] + alpha[q]) * psi_d(dU * dU + dV * dV, A.eps);
}

// planes of A.sys
enum { S_W1, S_W2, S_A12, S_B1, S_B2, S_GL, S_GR, S_GU, S_GD, S_NPLANES };

__global__ __launch_bounds__(256) void k_var_weights(VarArgs A, const float* __restrict__ du,
                                                     const float* __restrict__ dv) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    const int W = A.W, H = A.H;
    const int x = (int)(i % W), y = (int)(i / W);
    float JC[6], JG[6];
    for (int k = 0; k < 6; ++k) {
        JC[k] = A.coef[(long long)k * A.HW + i];
        JG[k] = A.coef[(long long)(6 + k) * A.HW + i];
    }
    const float dui = du[i], dvi = dv[i];
    const float wc = A.delta * psi_d(quad(JC, dui, dvi), A.eps);
    const float wg = A.gamma * psi_d(quad(JG, dui, dvi), A.eps);
    const float a11 = wc * JC[0] + wg * JG[0];
    const float a12 = wc * JC[1] + wg * JG[1];
    const float a22 = wc * JC[2] + wg * JG[2];
    float b1 = -(wc * JC[3] + wg * JG[3]);
    float b2 = -(wc * JC[4] + wg * JG[4]);
    // the 4 edges (0 where there is no neighbour) and the fixed part of the
    // neighbour sums, sum_j g (u0_j - u0_i)
    const float gl = x > 0 ? edge_weight(A, du, dv, i - 1, i) : 0.0f;
    const float gr = x + 1 < W ? edge_weight(A, du, dv, i, i + 1) : 0.0f;
    const float gu = y > 0 ? edge_weight(A, du, dv, i - W, i) : 0.0f;
    const float gd = y + 1 < H ? edge_weight(A, du, dv, i, i + W) : 0.0f;
    const float u0i = A.u0[2 * i], v0i = A.u0[2 * i + 1];
    auto fold = [&](float g, long long j) {
        b1 += g * (A.u0[2 * j] - u0i);
        b2 += g * (A.u0[2 * j + 1] - v0i);
    };
    if (x > 0) fold(gl, i - 1);
    if (x + 1 < W) fold(gr, i + 1);
    if (y > 0) fold(gu, i - W);
    if (y + 1 < H) fold(gd, i + W);
    const float sw = ((gl + gr) + gu) + gd;
    float* P = A.sys;
    const long long HW = A.HW;
    // omega over the diagonal (0 for an empty equation, which keeps its
    // unknown)
    const float d1 = a11 + sw, d2 = a22 + sw;
    P[S_W1 * HW + i] = d1 > 0.0f ? A.omega / d1 : 0.0f;
    P[S_W2 * HW + i] = d2 > 0.0f ? A.omega / d2 : 0.0f;
    P[S_A12 * HW + i] = a12;
    P[S_B1 * HW + i] = b1;
    P[S_B2 * HW + i] = b2;
    P[S_GL * HW + i] = gl;
    P[S_GR * HW + i] = gr;
    P[S_GU * HW + i] = gu;
    P[S_GD * HW + i] = gd;
}

#ifndef EPIC_VAR_TX
#define EPIC_VAR_TX 64
#endif
#ifndef EPIC_VAR_TY
#define EPIC_VAR_TY 32
#endif
#ifndef EPIC_VAR_S
#define EPIC_VAR_S 12
#endif
#ifndef EPIC_VAR_NT
#define EPIC_VAR_NT 512
#endif

// Tile TX x TY, halo S (= the most half-sweeps a launch runs; even, so every
// launch starts with red), NT threads.  The region RX x RY = (TX + 2S) x
// (TY + 2S) holds RX/2 pixels of each colour per row; slot s of colour c
// in region row y is the pixel x = 2s + ((c + X0 + Y0 + y) & 1).  In LDS
// each colour is a padded (RY + 2) x (RX/2 + 2) array of (du, dv): the
// neighbours of slot s (colour c, row y, parity p) are, in the other
// colour's array, slots s - 1 + p and s + p of row y and slot s of rows
// y - 1 and y + 1 -- consecutive lanes read consecutive words.
template <int TX, int TY, int S, int NT>
__global__ __launch_bounds__(NT) void k_var_sor(VarArgs A, const float* __restrict__ du_in,
                                                const float* __restrict__ dv_in, float* __restrict__ du_out,
                                                float* __restrict__ dv_out, int nh) {
    static_assert(S % 2 == 0 && TX % 2 == 0, "even halo and tile width");
    constexpr int RX = TX + 2 * S, RY = TY + 2 * S, RXh = RX / 2, NS = RY * RXh;
    constexpr int KP = (NS + NT - 1) / NT;
    constexpr int LW = RXh + 2, LN = (RY + 2) * LW;
    __shared__ float2 L[2][LN];
    const int tid = threadIdx.x;
    const int W = A.W, H = A.H;
    const long long HW = A.HW;
    const int tiles_x = (W + TX - 1) / TX;
    const int X0 = (int)(blockIdx.x % tiles_x) * TX - S, Y0 = (int)(blockIdx.x / tiles_x) * TY - S;
    for (int k = tid; k < 2 * LN; k += NT) (&L[0][0])[k] = make_float2(0.0f, 0.0f);
    __syncthreads();
    // this thread's slots: the 9 numbers, its own (du, dv), the LDS cells
    float cf[2][KP][S_NPLANES];
    float2 own[2][KP];
    int cell[2][KP], par[2][KP];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int slot = tid + k * NT;
            const int y = slot / RXh, s = slot % RXh;
            const int p = (c + X0 + Y0 + y) & 1;
            const int gx = X0 + 2 * s + p, gy = Y0 + y;
            // slots past the region park on a harmless cell (they never
            // update: W = 0, and their writes are skipped)
            cell[c][k] = slot < NS ? (y + 1) * LW + s + 1 : LW + 1;
            par[c][k] = p;
            own[c][k] = make_float2(0.0f, 0.0f);
#pragma unroll
            for (int q = 0; q < S_NPLANES; ++q) cf[c][k][q] = 0.0f;   // W = 0: never updated
            if (slot < NS && gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const long long i = (long long)gy * W + gx;
#pragma unroll
                for (int q = 0; q < S_NPLANES; ++q) cf[c][k][q] = A.sys[q * HW + i];
                own[c][k] = make_float2(du_in[i], dv_in[i]);
                L[c][cell[c][k]] = own[c][k];
            }
        }
    }
    __syncthreads();
    const float om1 = 1.0f - A.omega;
    // one half-sweep over colour C (a compile-time colour: the register
    // arrays are indexed by constants only)
    auto half = [&](auto colour) {
        constexpr int c = decltype(colour)::value;
        const float2* N = L[c ^ 1];
        // all neighbour reads first (this half-sweep writes only colour c),
        // so the reads of every slot are in flight together
        float2 nb[KP][4];
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int e = cell[c][k], p = par[c][k];
            nb[k][0] = N[e - 1 + p];
            nb[k][1] = N[e + p];
            nb[k][2] = N[e - LW];
            nb[k][3] = N[e + LW];
        }
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const float* f = cf[c][k];
            const float2 l = nb[k][0], r = nb[k][1], u = nb[k][2], d = nb[k][3];
            // every rounding spelled out, so the result does not depend on
            // how the compiler schedules (and fuses) the unrolled slots:
            // any tiling gives the same bits
            const float su = __fmaf_rn(f[S_GD], d.x, __fmaf_rn(f[S_GU], u.x, __fmaf_rn(f[S_GR], r.x,
                                                                                        __fmul_rn(f[S_GL], l.x))));
            const float sv = __fmaf_rn(f[S_GD], d.y, __fmaf_rn(f[S_GU], u.y, __fmaf_rn(f[S_GR], r.y,
                                                                                        __fmul_rn(f[S_GL], l.y))));
            float2 v = own[c][k];
            if (f[S_W1] > 0.0f)
                v.x = __fmaf_rn(__fadd_rn(__fmaf_rn(-f[S_A12], v.y, f[S_B1]), su), f[S_W1], __fmul_rn(om1, v.x));
            if (f[S_W2] > 0.0f)
                v.y = __fmaf_rn(__fadd_rn(__fmaf_rn(-f[S_A12], v.x, f[S_B2]), sv), f[S_W2], __fmul_rn(om1, v.y));
            own[c][k] = v;
        }
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if (tid + k * NT < NS) L[c][cell[c][k]] = own[c][k];
        __syncthreads();
    };
    for (int h = 0; h < nh; h += 2) {     // nh is even: red, then black
        half(std::integral_constant<int, 0>{});
        half(std::integral_constant<int, 1>{});
    }
    // the tile (distance >= S from the region's edge) is exact
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int slot = tid + k * NT;
            const int y = slot / RXh, s = slot % RXh;
            const int x = 2 * s + par[c][k];
            const int gx = X0 + x, gy = Y0 + y;
            if (slot < NS && x >= S && x < S + TX && y >= S && y < S + TY && gx < W && gy < H) {
                const long long i = (long long)gy * W + gx;
                du_out[i] = own[c][k].x;
                dv_out[i] = own[c][k].y;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_var_out(VarArgs A, const float* __restrict__ du,
                                                 const float* __restrict__ dv) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.HW) return;
    A.flow[2 * i] = A.u0[2 * i] + du[i];
    A.flow[2 * i + 1] = A.u0[2 * i + 1] + dv[i];
}

__global__ __launch_bounds__(256) void k_var_zero(float* __restrict__ du, float* __restrict__ dv, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    du[i] = 0.0f;
    dv[i] = 0.0f;
}

hipError_t launch_variational(const VarArgs& A, hipStream_t s) {
    constexpr int TX = EPIC_VAR_TX, TY = EPIC_VAR_TY, S = EPIC_VAR_S, NT = EPIC_VAR_NT;
    const dim3 g((unsigned)((A.HW + 255) / 256)), b(256);
    const unsigned tiles = (unsigned)(((A.W + TX - 1) / TX) * ((A.H + TY - 1) / TY));
    int cur = 0;
    hipLaunchKernelGGL(k_var_zero, g, b, 0, s, A.du[0], A.dv[0], A.HW);
    hipLaunchKernelGGL(k_var_warp, g, b, 0, s, A);
    hipLaunchKernelGGL(k_var_coef, g, b, 0, s, A);
    for (int f = 0; f < A.fixed_point; ++f) {
        hipLaunchKernelGGL(k_var_weights, g, b, 0, s, A, A.du[cur], A.dv[cur]);
        for (int h = 0; h < 2 * A.sor; h += S) {
            const int nh = 2 * A.sor - h < S ? 2 * A.sor - h : S;
            hipLaunchKernelGGL((k_var_sor<TX, TY, S, NT>), dim3(tiles), dim3(NT), 0, s, A, A.du[cur], A.dv[cur],
                               A.du[cur ^ 1], A.dv[cur ^ 1], nh);
            cur ^= 1;
        }
    }
    hipLaunchKernelGGL(k_var_out, g, b, 0, s, A, A.du[cur], A.dv[cur]);
    return hipGetLastError();
}

}  // namespace epic
