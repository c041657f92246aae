// k_image_cost.hip -- the cost map from the image gradient: C(p) =
// ||grad I(p)||_2 + eps (Table 2 of the paper, the norm-of-gradient contour
// row; Sec. 4 uses the same gradient norm for its smoothness weight).  The
// gradient is taken by central differences, (I(x+1) - I(x-1)) / 2 and
// (I(y+1) - I(y-1)) / 2, with the border pixel repeated outside the image,
// and the norm runs over both directions and all channels (interleaved,
// 1 to 4 per pixel).
//
// A streaming stencil bound by HBM: 4*ch bytes read and 4 written per
// pixel.  One thread per pixel, a workgroup per 64 x 4 pixel tile (a
// wavefront per 64-pixel row segment): the left and right neighbours a
// thread reads are its lanes' pixels, fetched once for the wavefront, and
// the rows above and below are read again by the neighbouring tiles while
// they are still in the L2 or the Infinity Cache.  Measured against a
// 4096 x 4572 RGB image, this simple form outran strips walked down by one
// workgroup with the rows in registers and the neighbours in LDS (every
// row then waits for its loads in turn).  FP32, one rounding per
// operation.
#include "epic_dev.h"

namespace epic {

namespace {

constexpr int kTileW = 64, kTileH = 4;     // pixels per workgroup

template <int CH>
__device__ __forceinline__ void load_px(const float* img, long long i, float (&v)[CH]) {
    const EPIC_GLOBAL float* g = gmem(img) + i * CH;
#pragma unroll
    for (int c = 0; c < CH; ++c) v[c] = g[c];
}

}  // namespace

template <int CH>
__global__ __launch_bounds__(kTileW * kTileH) void k_image_cost(ImageCostArgs args) {
    // one rounding per operation (no fused multiply-adds)
#pragma clang fp contract(off)
    // the image whose tiles this block belongs to: a binary search over the
    // ascending block bases (a block's whole work is a few loads, so a
    // linear walk over up to 32 images would take as long as the loads)
    const int im = find_pair(args.n, (int)blockIdx.x, [&](int i) { return args.img[i].block_base; });
    const ImageDesc& D = args.img[im];
    const int H = D.H, W = D.W;
    const int tx = (W + kTileW - 1) / kTileW;
    const int b = (int)blockIdx.x - D.block_base;
    const int x = (b % tx) * kTileW + (int)(threadIdx.x % kTileW);
    const int y = (b / tx) * kTileH + (int)(threadIdx.x / kTileW);
    if (x >= W || y >= H) return;
    // neighbours, the border pixel repeated outside the image
    const int xl = max(x - 1, 0), xr = min(x + 1, W - 1), yu = max(y - 1, 0), yd = min(y + 1, H - 1);
    float l[CH], r[CH], u[CH], d[CH];
    load_px<CH>(D.image, (long long)y * W + xl, l);
    load_px<CH>(D.image, (long long)y * W + xr, r);
    load_px<CH>(D.image, (long long)yu * W + x, u);
    load_px<CH>(D.image, (long long)yd * W + x, d);
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const float gx = 0.5f * (r[c] - l[c]);
        const float gy = 0.5f * (d[c] - u[c]);
        s = s + (gx * gx + gy * gy);
    }
    gmem(D.cost)[(long long)y * W + x] = __fsqrt_rn(s) + args.eps;
}

int image_cost_blocks(int H, int W) {
    return ((W + kTileW - 1) / kTileW) * ((H + kTileH - 1) / kTileH);
}

hipError_t launch_image_cost(const ImageCostArgs& args, int channels, int total_blocks, hipStream_t s) {
    switch (channels) {
        case 1: hipLaunchKernelGGL(k_image_cost<1>, dim3(total_blocks), dim3(kTileW * kTileH), 0, s, args); break;
        case 2: hipLaunchKernelGGL(k_image_cost<2>, dim3(total_blocks), dim3(kTileW * kTileH), 0, s, args); break;
        case 3: hipLaunchKernelGGL(k_image_cost<3>, dim3(total_blocks), dim3(kTileW * kTileH), 0, s, args); break;
        case 4: hipLaunchKernelGGL(k_image_cost<4>, dim3(total_blocks), dim3(kTileW * kTileH), 0, s, args); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace epic
