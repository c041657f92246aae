// k_exact.hip -- the exact per-pixel geodesic interpolation (Table 2 of the
// paper, the "Geodesic (exact)" row; Sec. 5.2 compares it with the
// approximation of Sec. 3.4): every pixel p gets its own K nearest matches
// under the geodesic distance of Eq. (3) itself, D_G(p, p_m), ordered by
// (distance, index), with weights exp(-a D_G), and its own NW or LA
// estimate evaluated at p -- no Voronoi cells, no match graph.
//
// The distances come from single-source transforms: each match is a pair of
// its own in a batch (the same cost map, that one match) run through the
// tiled transform of k_geodesic.hip in FP32.  The approximated interpolation
// runs first and bounds, at every pixel, the distance of its K-th nearest
// match (k_exact_bound); the transforms keep only distances within those
// bounds, which is exact: a pixel on a shortest path from one of p's K
// nearest matches to p has that match among its own K nearest, so the path
// is never cut.  Sources are processed in chunks that fit the workspace;
// after each chunk, k_exact_select folds the chunk's distances into every
// pixel's K smallest (distance, index) keys.  k_exact_owner first marks the
// matches that hold their pixel (placed, lowest index), so dropped and
// duplicate matches never enter a list.  k_exact_fit then fits each pixel
// (fit.h) with the pixel as the anchor.
#include "epic_dev.h"
#include "fit.h"
#include "wave.h"

namespace epic {

// Per pixel p, an upper bound of the distance of its K-th nearest match:
// D(p) + the K-th graph distance from p's cell's match (the approximation
// of Eq. (4) is the length of a path of the pixel graph for each of those K
// matches, so K matches lie within it).  Widened by 1e-3 relative (and
// 1e-6) so that rounding in either sum never makes it too small; infinite
// (no bound) when the cell has fewer than K neighbours in its list or the
// approximated pass reported a problem.
__global__ __launch_bounds__(256) void k_exact_bound(const PairDev* __restrict__ full, ExactArgs A) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= A.HW) return;
    const PairDev& P = full[0];
    float u = __int_as_float(0x7f800000);
    const bool ok = P.counters[C_STATUS] == 0 && (P.counters[C_OVERFLOW] & 2) == 0;
    const u64 k = P.keys[p];
    const u32 L = key_label(k);
    if (ok && L < (u32)P.N) {
        const long long j = (long long)L * A.K + (A.K - 1);
        if (A.knn_idx[j] >= 0) u = (key_dist(k) + A.knn_d[j]) * 1.001f + 1e-6f;
    }
    A.ubound[p] = u;
}

__global__ __launch_bounds__(256) void k_exact_owner(const PairDev* __restrict__ full, ExactArgs A) {
    const int m = (int)(blockIdx.x * 256 + threadIdx.x);
    if (m >= A.N) return;
    const PairDev& P = full[0];
    const int sp = P.seed_pix[m];
    A.owner[m] = (sp >= 0 && key_label(P.keys[sp]) == (u32)m) ? 1 : 0;
}

// The pixel box each source of a chunk reached (its bounded transform
// recorded the tiles): for the selection (sources that hold no pixel count
// as reaching nothing) and for the next chunk's clearing of the same
// workspace; empty boxes have x0 > x1.
__global__ __launch_bounds__(256) void k_exact_boxes(const PairDev* __restrict__ chunk, int nsrc, int src0,
                                                     ExactArgs A) {
    const int j = (int)(blockIdx.x * 256 + threadIdx.x);
    if (j >= nsrc) return;
    const int* c = chunk[j].counters;
    int4 b = make_int4(0x7fffffff, 0, -1, -1);
    if (c[C_BX1] > 0) {
        b.x = ((1 << 24) - c[C_BX0]) * 32;
        b.y = ((1 << 24) - c[C_BY0]) * 16;
        b.z = min((c[C_BX1] - 1) * 32 + 31, A.W - 1);
        b.w = min((c[C_BY1] - 1) * 16 + 15, A.H - 1);
    }
    A.clear_boxes[j] = b;
    if (A.owner[src0 + j] == 0) b = make_int4(0x7fffffff, 0, -1, -1);
    A.boxes[j] = b;
}

// One wavefront per 64 consecutive pixels (a pixel per lane); each lane
// keeps its K smallest (distance bits << 32 | match) keys as a max-heap in
// LDS, entry k of lane l at [k * 64 + l] (consecutive lanes, consecutive
// words; 64 KiB at K = 128), held in the workspace between chunks in heap
// order and sorted ascending by the last chunk (keys are distinct, so the
// K smallest and their order are the (distance, index) order whatever the
// heap's shape).  The wavefront first lists the chunk's sources whose box
// meets its pixels, then reads only their distances.
__global__ __launch_bounds__(64) void k_exact_select(const PairDev* __restrict__ chunk, int nsrc, int src0,
                                                     int first, int last, ExactArgs A) {
    extern __shared__ u64 L[];
    unsigned short* hits = reinterpret_cast<unsigned short*>(L + (size_t)A.K * 64);   // up to kExactChunk
    const int lane = threadIdx.x;
    const long long p0 = (long long)blockIdx.x * 64, p = p0 + lane;
    const bool valid = p < A.HW;
    const int K = A.K;
    auto H = [&](int k) -> u64& { return L[k * 64 + lane]; };
    int cnt = 0;
    for (int k = 0; k < K; ++k) {
        const u64 v = (!first && valid) ? gmem(A.lists)[(long long)k * A.HW + p] : ~0ull;
        H(k) = v;
        cnt += v != ~0ull ? 1 : 0;          // the heap fills [0, cnt)
    }
    // the wavefront's pixels: rows ya..yb, columns xa..xb (all of them when
    // the run wraps a row)
    const long long pe = min(p0 + 63, A.HW - 1);
    const int ya = (int)(p0 / A.W), yb = (int)(pe / A.W);
    const int xa = ya == yb ? (int)(p0 % A.W) : 0, xb = ya == yb ? (int)(pe % A.W) : A.W - 1;
    int nh = 0;
    for (int j0 = 0; j0 < nsrc; j0 += 64) {
        const int j = j0 + lane;
        bool hit = false;
        if (j < nsrc) {
            const int4 b = A.boxes[j];
            hit = b.x <= xb && b.z >= xa && b.y <= yb && b.w >= ya;
        }
        const u64 m = wave::ballot(hit);
        if (hit) hits[nh + wave::lanes_below(m)] = (unsigned short)j;
        nh += __popcll(m);
    }
    __syncthreads();
    // the listed sources in groups of 8 with all their loads in flight together
    constexpr int G = 8;
    for (int h0 = 0; h0 < nh; h0 += G) {
        float d[G];
        int jj[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            jj[u] = h0 + u < nh ? hits[h0 + u] : -1;                        // uniform
            d[u] = (jj[u] >= 0 && valid) ? key_dist(gmem(chunk[jj[u]].keys)[p]) : __int_as_float(0x7f800000);
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            if (!(d[u] < __int_as_float(0x7f800000))) continue;
            const u64 key = ((u64)__float_as_uint(d[u]) << 32) | (u32)(src0 + jj[u]);
            if (cnt < K) {
                // append and sift up
                int i = cnt++;
                while (i > 0) {
                    const int up = (i - 1) >> 1;
                    const u64 pv = H(up);
                    if (!(pv < key)) break;
                    H(i) = pv;
                    i = up;
                }
                H(i) = key;
            } else if (key < H(0)) {
                // replace the largest and sift down
                int i = 0;
                for (;;) {
                    const int l = 2 * i + 1;
                    if (l >= K) break;
                    int c = l;
                    u64 cv = H(l);
                    if (l + 1 < K) {
                        const u64 rv = H(l + 1);
                        if (rv > cv) {
                            c = l + 1;
                            cv = rv;
                        }
                    }
                    if (!(cv > key)) break;
                    H(i) = cv;
                    i = c;
                }
                H(i) = key;
            }
        }
    }
    if (last) {
        // heapsort into ascending order
        for (int end = cnt - 1; end > 0; --end) {
            const u64 top = H(0), key = H(end);
            H(end) = top;
            int i = 0;
            for (;;) {
                const int l = 2 * i + 1;
                if (l >= end) break;
                int c = l;
                u64 cv = H(l);
                if (l + 1 < end) {
                    const u64 rv = H(l + 1);
                    if (rv > cv) {
                        c = l + 1;
                        cv = rv;
                    }
                }
                if (!(cv > key)) break;
                H(i) = cv;
                i = c;
            }
            H(i) = key;
        }
    }
    if (valid)
        for (int k = 0; k < K; ++k) gmem(A.lists)[(long long)k * A.HW + p] = H(k);
}

// One wavefront per pixel: its list, two entries per lane at most, the
// neighbours' rows, and the fit about the pixel (displacements taken
// relative to the nearest neighbour's).
template <int KMAX>
__global__ __launch_bounds__(64) void k_exact_fit(ExactArgs A) {
    constexpr int RK = KMAX / 64;
    const int lane = threadIdx.x;
    const long long p = blockIdx.x;
    const int K = A.K;
    int node[RK];
    float kd[RK];
    int n = 0;
#pragma unroll
    for (int r = 0; r < RK; ++r) {
        const int j = lane + 64 * r;
        const u64 v = j < K ? gmem(A.lists)[(long long)j * A.HW + p] : ~0ull;
        node[r] = v != ~0ull ? (int)(u32)v : -1;
        kd[r] = v != ~0ull ? key_dist(v) : 0.0f;
        n += __popcll(wave::ballot(node[r] >= 0));
    }
    float2 f;
    if (n == 0) {
        f.x = f.y = __int_as_float(0x7fc00000);          // no match in the image
    } else {
        const int n0 = __builtin_amdgcn_readfirstlane(node[0]);
        float4 mrow[RK];
#pragma unroll
        for (int r = 0; r < RK; ++r) mrow[r] = gload(reinterpret_cast<const float4*>(A.matches) + (node[r] >= 0 ? node[r] : n0));
        const float4 m0 = gload(reinterpret_cast<const float4*>(A.matches) + n0);
        const float xp = (float)(int)(p % A.W), yp = (float)(int)(p / A.W);
        const FitOut fo = fit_about<RK, false>(lane, n, kd, mrow, xp, yp, m0.z - m0.x, m0.w - m0.y,
                                               (double)m0.z - (double)m0.x, (double)m0.w - (double)m0.y,
                                               A.a, A.wpow, A.mode == 1, A.fp64_route, A.deg_tau);
        f.x = fo.p[4];
        f.y = fo.p[5];
    }
    if (lane == 0) gstore(reinterpret_cast<float2*>(A.flow) + p, f);
}

hipError_t launch_exact_owner(const PairDev* full, const ExactArgs& A, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_owner, dim3((A.N + 255) / 256), dim3(256), 0, s, full, A);
    return hipGetLastError();
}

hipError_t launch_exact_select(const PairDev* chunk, int nsrc, int src0, int first, int last, const ExactArgs& A,
                               hipStream_t s) {
    if (nsrc > kExactChunk) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_exact_boxes, dim3((unsigned)((nsrc + 255) / 256)), dim3(256), 0, s, chunk, nsrc, src0, A);
    const size_t lds = (size_t)A.K * 64 * sizeof(u64) + (size_t)kExactChunk * sizeof(unsigned short);
    if (lds > 65536) {
        // above the default dynamic LDS limit of a launch (K > 124)
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_exact_select),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_exact_select, dim3((unsigned)((A.HW + 63) / 64)), dim3(64), lds, s, chunk, nsrc, src0,
                       first, last, A);
    return hipGetLastError();
}

hipError_t launch_exact_bound(const PairDev* full, const ExactArgs& A, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_bound, dim3((unsigned)((A.HW + 255) / 256)), dim3(256), 0, s, full, A);
    return hipGetLastError();
}

hipError_t launch_exact_fit(const ExactArgs& A, hipStream_t s) {
    const dim3 g((unsigned)A.HW);
    if (A.K <= 64) hipLaunchKernelGGL(k_exact_fit<64>, g, dim3(64), 0, s, A);
    else hipLaunchKernelGGL(k_exact_fit<128>, g, dim3(64), 0, s, A);
    return hipGetLastError();
}

}  // namespace epic
