// k_assign.hip -- dense assignment (Algorithm 1, steps 7-8; Sec. 3.4,
// "Piecewise field"): every pixel takes the model of its geodesic Voronoi
// cell, flow(p) = B_m (p - p_m) + c_m with m = L(p).  NW models have B = 0,
// so the field is piecewise constant for NW and piecewise affine for LA.
// Pixels of an image without any usable match get NaN.
//
// In the FP64 path the models are read in double and the flow is rounded to
// float at the end.
// Also: k_unpack splits the packed (D, label) keys for the debug entry point.
#include "epic_dev.h"

namespace epic {

namespace {

// Flow of pixel (x, y) with model m (NaN without a label).
__device__ __forceinline__ float2 assign_px(const PairDev& P, u32 m, int x, int y) {
    float2 f;
    if (m == NO_LABEL) {
        f.x = f.y = __int_as_float(0x7fc00000);
    } else if (P.params64) {
        const EPIC_GLOBAL double* B = gmem(P.params64) + 6LL * m;
        const double dx = (double)x - (double)gmem(P.matches)[4LL * m];
        const double dy = (double)y - (double)gmem(P.matches)[4LL * m + 1];
        f.x = (float)(B[0] * dx + B[1] * dy + B[4]);
        f.y = (float)(B[2] * dx + B[3] * dy + B[5]);
    } else {
        // a model is 24 bytes in a 256-byte aligned array: three 8-byte loads
        const float2* B = reinterpret_cast<const float2*>(P.params + 6LL * m);
        const float2 b01 = gload(B), b23 = gload(B + 1), c = gload(B + 2);
        const float2 pm = gload(reinterpret_cast<const float2*>(P.matches + 4LL * m));
        const float dx = (float)x - pm.x, dy = (float)y - pm.y;
        f.x = b01.x * dx + b01.y * dy + c.x;
        f.y = b23.x * dx + b23.y * dy + c.y;
    }
    return f;
}

}  // namespace

// PPT consecutive pixels per thread (row-major, a run may wrap to the next
// row).  With PPT > 1 the labels of a run are loaded together (16-byte loads
// of packed keys on the FP32 path) and its flow is stored as 16-byte pairs
// when the output allows it, so each wavefront keeps more memory requests in
// flight; that pays when the call has more pixels than the chip holds
// wavefronts of single pixels, and costs latency when it has fewer.
template <int PPT>
__global__ __launch_bounds__(PIX_BLOCK) void k_assign(const PairDev* __restrict__ pairs, RunDev run) {
    // the pair's blocks start at pix_block_base / PPT (a whole number: pixel
    // grids give each pair a multiple of ASSIGN_PPT blocks)
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].pix_block_base / PPT; });
    const PairDev& P = pairs[p];
    // H * W < 2^31 (checked on the host): 32-bit index arithmetic
    const u32 HW = (u32)P.W * (u32)P.H;
    const u32 i0 = ((u32)((int)blockIdx.x - P.pix_block_base / PPT) * PIX_BLOCK + threadIdx.x) * PPT;
    if (i0 >= HW || P.flow == nullptr) return;
    const u32 W = (u32)P.W;
    const int n = (int)min((u32)PPT, HW - i0);
    u32 m[PPT];
    if (P.labels) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) m[j] = j < n ? gmem(P.labels)[i0 + j] : NO_LABEL;
    } else if (PPT > 1 && n == PPT) {
        // the keys array is 256-byte aligned and i0 a multiple of PPT
#pragma unroll
        for (int h = 0; h < PPT / 2; ++h) {
            const uint4 k2 = gload(reinterpret_cast<const uint4*>(P.keys + i0) + h);
            m[2 * h] = k2.x;          // label: the low word of each key
            m[2 * h + 1] = k2.z;
        }
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j) m[j] = j < n ? key_label(gmem(P.keys)[i0 + j]) : NO_LABEL;
    }
    int x = (int)(i0 % W), y = (int)(i0 / W);
    float2 f[PPT];
    if (P.params64) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            f[j] = assign_px(P, m[j], x, y);
            if (++x == (int)W) {
                x = 0;
                ++y;
            }
        }
    } else {
        // consecutive pixels mostly share a cell: the model stays in
        // registers and is fetched again only when the label changes (the
        // same arithmetic as assign_px)
        u32 mc = NO_LABEL;
        float2 b01 = make_float2(0.0f, 0.0f), b23 = b01, c = b01, pm = b01;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (m[j] != NO_LABEL && m[j] != mc) {
                mc = m[j];
                const float2* B = reinterpret_cast<const float2*>(P.params + 6LL * mc);
                b01 = gload(B);
                b23 = gload(B + 1);
                c = gload(B + 2);
                pm = gload(reinterpret_cast<const float2*>(P.matches + 4LL * mc));
            }
            if (m[j] == NO_LABEL) {
                f[j].x = f[j].y = __int_as_float(0x7fc00000);
            } else {
                const float dx = (float)x - pm.x, dy = (float)y - pm.y;
                f[j].x = b01.x * dx + b01.y * dy + c.x;
                f[j].y = b23.x * dx + b23.y * dy + c.y;
            }
            if (++x == (int)W) {
                x = 0;
                ++y;
            }
        }
    }
    float2* out = reinterpret_cast<float2*>(P.flow) + i0;
    if (PPT > 1 && n == PPT && (reinterpret_cast<uintptr_t>(P.flow) & 15u) == 0) {
#pragma unroll
        for (int h = 0; h < PPT / 2; ++h)
            gstore(reinterpret_cast<float4*>(out) + h, make_float4(f[2 * h].x, f[2 * h].y, f[2 * h + 1].x, f[2 * h + 1].y));
    } else {
#pragma unroll
        for (int j = 0; j < PPT; ++j)
            if (j < n) gstore(out + j, f[j]);
    }
}

__global__ __launch_bounds__(PIX_BLOCK) void k_unpack(const PairDev* __restrict__ pairs, RunDev run, float* D,
                                                      int* L) {
    const PairDev& P = pairs[0];
    const long long i = (long long)blockIdx.x * PIX_BLOCK + threadIdx.x;
    if (i >= (long long)P.W * P.H) return;
    const u64 k = P.keys[i];
    if (P.labels) {                 // FP64 path: D is written as double
        if (D) reinterpret_cast<double*>(D)[i] = dbits(k);
        if (L) L[i] = P.labels[i] == NO_LABEL ? -1 : (int)P.labels[i];
        return;
    }
    if (D) D[i] = key_dist(k);
    if (L) L[i] = key_label(k) == NO_LABEL ? -1 : (int)key_label(k);
}

hipError_t launch_assign(const PairDev* d_pairs, const RunDev& run, int pix_blocks, long long total_px,
                         hipStream_t s) {
    // 256 CUs x 32 wavefronts x 64 lanes: pixels of one full chip at one per thread
    constexpr long long kChipLanes = 256LL * 32 * 64;
    if (total_px >= (long long)ASSIGN_PPT * kChipLanes)
        hipLaunchKernelGGL(k_assign<ASSIGN_PPT>, dim3(pix_blocks / ASSIGN_PPT), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    else
        hipLaunchKernelGGL(k_assign<1>, dim3(pix_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

hipError_t launch_unpack(const PairDev* d_pairs, const RunDev& run, int total_blocks, float* D, int* L,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_unpack, dim3(total_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run, D, L);
    return hipGetLastError();
}

}  // namespace epic
