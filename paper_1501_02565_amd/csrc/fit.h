// fit.h -- one kernel-weighted fit about an anchor point, by one wavefront
// (Eq. 1 and Eq. 2 of the paper): the n nearest matches (distance d_j, row
// x, y, x', y') are held two per lane at most, lane + 64 r.
//
//   weights k = exp(-a d), w = k^2 (each equation of Eq. 2 scaled by k) or k
//   NW:  c = u_a + sum k (u - u_a) / sum k                       (B = 0)
//   LA:  B from the weighted normal equations of the positions centred
//        about their weighted centroid, c the displacement the fitted map
//        gives at the anchor
// Positions are taken relative to the anchor and displacements relative to
// u_a, so the sums stay small.  FP32 first; a neighbourhood whose FP32
// covariance has an eigenvalue ratio below fp64_route (or fewer than 3
// neighbours) is re-accumulated and solved in FP64, where a ratio at or
// below deg_tau is near-collinear and falls back to NW.  With F64 the FP64
// solve is the only one.  Sums are DPP wave reductions in a fixed order.
#pragma once

#include "epic_dev.h"
#include "wave.h"

namespace epic {

struct FitOut {
    float p[6];          // b00 b01 b10 b11 c0 c1 of u(x) = B (x - anchor) + c
    double p64[6];       // the same in double when the FP64 solve ran
    bool fp64;           // the FP64 solve ran
    bool degenerate;     // LA fell back to NW
};

template <int RK, bool F64, typename RT>
__device__ __forceinline__ FitOut fit_about(int lane, int n, const RT (&kdist)[RK], const float4 (&mrow)[RK],
                                            float xm, float ym, float um, float vm, double umd, double vmd,
                                            float a, int wpow, bool la, float fp64_route, double deg_tau) {
    FitOut fo;
    float* out = fo.p;
    for (int i = 0; i < 6; ++i) out[i] = 0.f;
    fo.degenerate = false;
    bool need64 = F64;
    if constexpr (!F64) {      // the FP64-everywhere path goes straight to FP64
        float dx[RK], dy[RK], du[RK], dv[RK], kk[RK], ww[RK];
        float tk = 0.f, tu = 0.f, tv = 0.f, sw = 0.f, sx = 0.f, sy = 0.f;
#pragma unroll
        for (int r = 0; r < RK; ++r) {
            const int j = lane + 64 * r;
            dx[r] = dy[r] = du[r] = dv[r] = kk[r] = ww[r] = 0.f;
            if (j < n) {
                const float dj = (float)kdist[r];
                const float4 mn = mrow[r];
                dx[r] = mn.x - xm;
                dy[r] = mn.y - ym;
                du[r] = (mn.z - mn.x) - um;
                dv[r] = (mn.w - mn.y) - vm;
                kk[r] = expf(-a * dj);
                ww[r] = wpow == 1 ? kk[r] : kk[r] * kk[r];
                tk += kk[r];
                tu += kk[r] * du[r];
                tv += kk[r] * dv[r];
                sw += ww[r];
                sx += ww[r] * dx[r];
                sy += ww[r] * dy[r];
            }
        }
        tk = wave::sum(tk);
        tu = wave::sum(tu);
        tv = wave::sum(tv);
        // one hardware reciprocal per distinct denominator (1 ulp; the
        // denominators are sums of weights >= 1, or a determinant whose
        // ill-conditioned cases go to FP64), then products
        const float itk = __builtin_amdgcn_rcpf(tk);
        out[4] = um + tu * itk;
        out[5] = vm + tv * itk;
        if (la) {
            sw = wave::sum(sw);
            sx = wave::sum(sx);
            sy = wave::sum(sy);
            const float isw = __builtin_amdgcn_rcpf(sw);
            const float mx = sx * isw, my = sy * isw;
            float sxx = 0.f, sxy = 0.f, syy = 0.f, sxu = 0.f, syu = 0.f, sxv = 0.f, syv = 0.f, su = 0.f, sv = 0.f;
#pragma unroll
            for (int r = 0; r < RK; ++r) {
                const float ex = dx[r] - mx, ey = dy[r] - my, w = ww[r];
                sxx += w * ex * ex;
                sxy += w * ex * ey;
                syy += w * ey * ey;
                sxu += w * ex * du[r];
                syu += w * ey * du[r];
                sxv += w * ex * dv[r];
                syv += w * ey * dv[r];
                su += w * du[r];
                sv += w * dv[r];
            }
            sxx = wave::sum(sxx); sxy = wave::sum(sxy); syy = wave::sum(syy);
            sxu = wave::sum(sxu); syu = wave::sum(syu); sxv = wave::sum(sxv); syv = wave::sum(syv);
            su = wave::sum(su); sv = wave::sum(sv);
            const float det = sxx * syy - sxy * sxy;
            const float tr = sxx + syy;
            const float disc = __builtin_amdgcn_sqrtf((sxx - syy) * (sxx - syy) + 4.0f * sxy * sxy);
            const float l1 = 0.5f * (tr + disc);
            const float ratio = l1 > 0.f ? det / (l1 * l1) : 0.f;
            need64 = n < 3 || !(ratio >= fp64_route);
            if (!need64) {
                const float idet = __builtin_amdgcn_rcpf(det);
                const float b00 = (syy * sxu - sxy * syu) * idet, b01 = (sxx * syu - sxy * sxu) * idet;
                const float b10 = (syy * sxv - sxy * syv) * idet, b11 = (sxx * syv - sxy * sxv) * idet;
                out[0] = b00; out[1] = b01; out[2] = b10; out[3] = b11;
                out[4] = um + su * isw - (b00 * mx + b01 * my);
                out[5] = vm + sv * isw - (b10 * mx + b11 * my);
            }
        }
    }
    fo.fp64 = need64;
    if (need64) {
        // FP64: re-accumulate from the inputs and solve (or fall back to NW)
        const double xmd = xm, ymd = ym;
        double Dx[RK], Dy[RK], Du[RK], Dv[RK], Dw[RK];
        double Tk = 0, Tu = 0, Tv = 0, Sw = 0, Sx = 0, Sy = 0;
#pragma unroll
        for (int r = 0; r < RK; ++r) {
            const int j = lane + 64 * r;
            Dx[r] = Dy[r] = Du[r] = Dv[r] = Dw[r] = 0.0;
            if (j < n) {
                const double dj = (double)kdist[r];
                const double x = mrow[r].x, y = mrow[r].y;
                Dx[r] = x - xmd;
                Dy[r] = y - ymd;
                Du[r] = ((double)mrow[r].z - x) - umd;
                Dv[r] = ((double)mrow[r].w - y) - vmd;
                const double k = exp(-(double)a * dj);
                Dw[r] = wpow == 1 ? k : k * k;
                Tk += k; Tu += k * Du[r]; Tv += k * Dv[r];
                Sw += Dw[r]; Sx += Dw[r] * Dx[r]; Sy += Dw[r] * Dy[r];
            }
        }
        Tk = wave::sum(Tk); Tu = wave::sum(Tu); Tv = wave::sum(Tv);
        double* o = fo.p64;
        o[0] = o[1] = o[2] = o[3] = 0.0;
        o[4] = umd + Tu / Tk;
        o[5] = vmd + Tv / Tk;
        if (la) {
            Sw = wave::sum(Sw); Sx = wave::sum(Sx); Sy = wave::sum(Sy);
            const double mx = Sx / Sw, my = Sy / Sw;
            double sxx = 0, sxy = 0, syy = 0, sxu = 0, syu = 0, sxv = 0, syv = 0, su = 0, sv = 0;
#pragma unroll
            for (int r = 0; r < RK; ++r) {
                const double ex = Dx[r] - mx, ey = Dy[r] - my, w = Dw[r];
                sxx += w * ex * ex; sxy += w * ex * ey; syy += w * ey * ey;
                sxu += w * ex * Du[r]; syu += w * ey * Du[r];
                sxv += w * ex * Dv[r]; syv += w * ey * Dv[r];
                su += w * Du[r]; sv += w * Dv[r];
            }
            sxx = wave::sum(sxx); sxy = wave::sum(sxy); syy = wave::sum(syy);
            sxu = wave::sum(sxu); syu = wave::sum(syu); sxv = wave::sum(sxv); syv = wave::sum(syv);
            su = wave::sum(su); sv = wave::sum(sv);
            // covariance normalised by the weight sum; eigenvalues l1 >= l2
            const double cxx = sxx / Sw, cxy = sxy / Sw, cyy = syy / Sw;
            const double tr = cxx + cyy;
            const double disc = sqrt((cxx - cyy) * (cxx - cyy) + 4.0 * cxy * cxy);
            const double l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
            fo.degenerate = n < 3 || !(l1 > 0.0) || l2 <= deg_tau * l1;
            if (!fo.degenerate) {
                const double det = sxx * syy - sxy * sxy;
                const double b00 = (syy * sxu - sxy * syu) / det, b01 = (sxx * syu - sxy * sxu) / det;
                const double b10 = (syy * sxv - sxy * syv) / det, b11 = (sxx * syv - sxy * sxv) / det;
                o[0] = b00; o[1] = b01; o[2] = b10; o[3] = b11;
                o[4] = umd + su / Sw - (b00 * mx + b01 * my);
                o[5] = vmd + sv / Sw - (b10 * mx + b11 * my);
            }
        }
        for (int i = 0; i < 6; ++i) out[i] = (float)o[i];
    }
    return fo;
}

}  // namespace epic
