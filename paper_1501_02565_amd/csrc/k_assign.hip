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

__global__ __launch_bounds__(PIX_BLOCK) void k_assign(const PairDev* __restrict__ pairs, RunDev run) {
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].pix_block_base; });
    const PairDev& P = pairs[p];
    // H * W < 2^31 (checked on the host): 32-bit index arithmetic
    const u32 i = (u32)((int)blockIdx.x - P.pix_block_base) * PIX_BLOCK + threadIdx.x;
    const u32 W = (u32)P.W;
    if (i >= W * (u32)P.H) return;
    const int px = (int)(i % W), py = (int)(i / W);
    const u32 m = P.labels ? gmem(P.labels)[i] : key_label(gmem(P.keys)[i]);
    float2 f;
    if (m == NO_LABEL) {
        f.x = f.y = __int_as_float(0x7fc00000);
    } else if (P.params64) {
        const EPIC_GLOBAL double* B = gmem(P.params64) + 6LL * m;
        const double dx = (double)px - (double)gmem(P.matches)[4LL * m];
        const double dy = (double)py - (double)gmem(P.matches)[4LL * m + 1];
        f.x = (float)(B[0] * dx + B[1] * dy + B[4]);
        f.y = (float)(B[2] * dx + B[3] * dy + B[5]);
    } else {
        const EPIC_GLOBAL float* B = gmem(P.params) + 6LL * m;
        const float2 pm = gload(reinterpret_cast<const float2*>(P.matches + 4LL * m));
        const float dx = (float)px - pm.x, dy = (float)py - pm.y;
        f.x = B[0] * dx + B[1] * dy + B[4];
        f.y = B[2] * dx + B[3] * dy + B[5];
    }
    gstore(reinterpret_cast<float2*>(P.flow) + i, f);
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

hipError_t launch_assign(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_assign, dim3(total_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

hipError_t launch_unpack(const PairDev* d_pairs, const RunDev& run, int total_blocks, float* D, int* L,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_unpack, dim3(total_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run, D, L);
    return hipGetLastError();
}

}  // namespace epic
