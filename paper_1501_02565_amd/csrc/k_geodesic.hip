// k_geodesic.hip -- geodesic distance transform and geodesic Voronoi labels.
//
// Computes, for every pixel p, D(p) = min over matches m of the geodesic
// distance D_G(p, p_m) of Eq. (3) and L(p) = the minimising match (lowest
// index on ties): the assignment map of Sec. 3.4 and the first term of the
// approximated distance, Eq. (4).  Eq. (3) is discretised on the 8-connected
// (or 4-connected) pixel graph; the step between adjacent pixels p, q costs
// len * (C(p) + C(q)) / 2 (trapezoid rule for the line integral of C).
//
// Algorithm (persistent, tile-asynchronous label-correcting relaxation):
//   * The image is cut into TW x TH tiles.  A tile is "dirty" when a pixel of
//     its 1-pixel halo may have improved since it was last processed.
//   * A fixed set of workgroups loops: claim a dirty tile (state 1 -> 2),
//     load it with its halo into LDS, relax every pixel from its neighbours
//     in place until nothing changes, write back the improved pixels, and
//     mark the neighbour tiles whose shared border changed as dirty.
//   * Each pixel's state is a packed (D, label) key, so relaxation is an
//     integer min: any relaxation order reaches the same fixpoint D (the
//     minimum over paths of the left-fold float sums); labels agree with
//     the lexicographic optimum except where rounded sums tie.
//   * `pending` counts dirty plus busy tiles; it is raised before a dirty
//     bit is set and lowered after a tile's neighbours were marked, so it is
//     zero only when the transform has converged.  Idle workers wait for it
//     with a wall-clock bound (error flag instead of a hang).
// Tile state bits: bit 0 dirty, bit 1 busy.
#include "epic_dev.h"

namespace epic {

namespace {

__device__ __forceinline__ u64 ld_key(const u64* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_key(u64* p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void mark_dirty(const RunDev& run, int t) {
    // raise pending first: it never under-counts dirty + busy tiles
    __hip_atomic_fetch_add(run.pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u32 old = __hip_atomic_fetch_or(&run.tile_state[t], 1u, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (old & 1u)
        __hip_atomic_fetch_add(run.pending, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

enum : int { B_L = 1, B_R = 2, B_T = 4, B_B = 8, B_TL = 16, B_TR = 32, B_BL = 64, B_BR = 128 };

}  // namespace

template <int TW, int TH, int CONN>
__global__ __launch_bounds__(256) void k_geodesic(const PairDev* __restrict__ pairs, RunDev run) {
    constexpr int NG = 256 / TW;       // row groups
    constexpr int PPT = TH / NG;       // pixels per thread (a vertical strip)
    constexpr int LW = TW + 2, LH = TH + 2;
    static_assert(NG * TW == 256 && PPT * NG == TH, "tile shape");
    __shared__ u64 sk[LH * LW];
    __shared__ float sc[LH * LW];
    __shared__ int s_tile, s_cand, s_border;

    constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    const int tid = threadIdx.x;
    const int lx = tid % TW, grp = tid / TW;
    const int total = run.total_tiles;
    int start = (int)(((long long)blockIdx.x * total) / gridDim.x);
    long long idle_since = wall_clock64();

    for (;;) {
        // ---------------------------------------------------- claim a tile
        if (tid == 0) s_cand = 0x7fffffff;
        __syncthreads();
        int found = 0x7fffffff;
        for (int i = tid; i < total; i += 256) {
            int t = start + i;
            if (t >= total) t -= total;
            if (__hip_atomic_load(&run.tile_state[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1u) {
                found = i;
                break;
            }
        }
        if (found != 0x7fffffff) atomicMin(&s_cand, found);
        __syncthreads();
        if (tid == 0) {
            int tile = -1;
            if (s_cand != 0x7fffffff) {
                int t = start + s_cand;
                if (t >= total) t -= total;
                u32 expect = 1u;
                if (__hip_atomic_compare_exchange_strong(&run.tile_state[t], &expect, 2u, __ATOMIC_ACQUIRE,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    tile = t;
            } else {
                const int pend = __hip_atomic_load(run.pending, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (pend <= 0) {
                    tile = -2;
                } else if (wall_clock64() - idle_since > run.spin_ticks) {
                    atomicOr(run.error, 1);
                    tile = -2;
                } else {
                    __builtin_amdgcn_s_sleep(8);
                }
            }
            s_tile = tile;
        }
        __syncthreads();
        const int tile = s_tile;
        if (tile == -2) return;
        if (tile < 0) continue;

        // ------------------------------------------------- load tile + halo
        const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
        const PairDev& P = pairs[p];
        const int lt = tile - P.tile_base;
        const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
        const int x0 = tx * TW, y0 = ty * TH, W = P.W, H = P.H;
        for (int i = tid; i < LH * LW; i += 256) {
            const int ly = i / LW, lxx = i - ly * LW;
            const int gx = x0 + lxx - 1, gy = y0 + ly - 1;
            u64 k = KEY_INF;
            float c = 0.0f;
            if (gx >= 0 && gy >= 0 && gx < W && gy < H) {
                const long long gi = (long long)gy * W + gx;
                k = ld_key(&P.keys[gi]);
                c = P.cost[gi];
            }
            sk[i] = k;
            sc[i] = c;
        }
        if (tid == 0) s_border = 0;
        __syncthreads();

        // ------------------------------------ own pixels and their step costs
        float wgt[PPT][CONN];
        u64 key[PPT], orig[PPT];
        bool valid[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int ly = grp * PPT + j;
            const int ci = (ly + 1) * LW + lx + 1;
            valid[j] = (x0 + lx < W) && (y0 + ly < H);
            const float cp = sc[ci];
#pragma unroll
            for (int k = 0; k < CONN; ++k) {
                const int gx = x0 + lx + DX[k], gy = y0 + ly + DY[k];
                const bool in = gx >= 0 && gy >= 0 && gx < W && gy < H;
                const float half = 0.5f * (cp + sc[ci + DY[k] * LW + DX[k]]);
                const float len = (k < 4) ? 1.0f : 1.41421356237309515f;
                wgt[j][k] = in ? len * half : __int_as_float(0x7f800000);
            }
            key[j] = orig[j] = sk[ci];
        }

        // ---------------------------------------- relax to a local fixpoint
        const int iter_cap = TW * TH + 8;
        for (int it = 0;; ++it) {
            int changed = 0;
            if ((it & 1) == 0) {
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const int ci = (grp * PPT + j + 1) * LW + lx + 1;
                    u64 best = key[j];
#pragma unroll
                    for (int k = 0; k < CONN; ++k) {
                        const u64 kq = sk[ci + DY[k] * LW + DX[k]];
                        const u64 cand = make_key(key_dist(kq) + wgt[j][k], key_label(kq));
                        best = cand < best ? cand : best;
                    }
                    if (valid[j] && best < key[j]) {
                        key[j] = best;
                        sk[ci] = best;
                        changed = 1;
                    }
                }
            } else {
#pragma unroll
                for (int jj = 0; jj < PPT; ++jj) {
                    const int j = PPT - 1 - jj;
                    const int ci = (grp * PPT + j + 1) * LW + lx + 1;
                    u64 best = key[j];
#pragma unroll
                    for (int k = 0; k < CONN; ++k) {
                        const u64 kq = sk[ci + DY[k] * LW + DX[k]];
                        const u64 cand = make_key(key_dist(kq) + wgt[j][k], key_label(kq));
                        best = cand < best ? cand : best;
                    }
                    if (valid[j] && best < key[j]) {
                        key[j] = best;
                        sk[ci] = best;
                        changed = 1;
                    }
                }
            }
            if (!__syncthreads_or(changed)) break;
            if (it > iter_cap) {
                if (tid == 0) atomicOr(run.error, 2);
                break;
            }
        }

        // ------------------------------------------- write back, find borders
        const int twe = min(TW, W - x0), the = min(TH, H - y0);
        int bm = 0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (valid[j] && key[j] != orig[j]) {
                const int ly = grp * PPT + j;
                st_key(&P.keys[(long long)(y0 + ly) * W + x0 + lx], key[j]);
                const bool l = lx == 0, r = lx == twe - 1, t = ly == 0, b = ly == the - 1;
                bm |= (l ? B_L : 0) | (r ? B_R : 0) | (t ? B_T : 0) | (b ? B_B : 0) |
                      ((l && t) ? B_TL : 0) | ((r && t) ? B_TR : 0) | ((l && b) ? B_BL : 0) |
                      ((r && b) ? B_BR : 0);
            }
        }
        if (bm) atomicOr(&s_border, bm);
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            const int b = s_border;
            const int nx = P.tiles_x, ny = P.tiles_y, base = P.tile_base;
            auto mark = [&](int cx, int cy) {
                if (cx >= 0 && cy >= 0 && cx < nx && cy < ny) mark_dirty(run, base + cy * nx + cx);
            };
            if (b & B_L) mark(tx - 1, ty);
            if (b & B_R) mark(tx + 1, ty);
            if (b & B_T) mark(tx, ty - 1);
            if (b & B_B) mark(tx, ty + 1);
            if (CONN == 8) {
                if (b & B_TL) mark(tx - 1, ty - 1);
                if (b & B_TR) mark(tx + 1, ty - 1);
                if (b & B_BL) mark(tx - 1, ty + 1);
                if (b & B_BR) mark(tx + 1, ty + 1);
            }
            __hip_atomic_fetch_and(&run.tile_state[tile], ~2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(run.pending, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            atomicAdd(&P.counters[C_TILE_VISITS], 1);
        }
        start = tile + 1 < total ? tile + 1 : 0;
        idle_since = wall_clock64();
    }
}

namespace {
template <int TW, int TH, int CONN>
hipError_t launch_t(const PairDev* d_pairs, const RunDev& run, int workers, hipStream_t s) {
    hipLaunchKernelGGL((k_geodesic<TW, TH, CONN>), dim3(workers), dim3(256), 0, s, d_pairs, run);
    return hipGetLastError();
}
template <int TW, int TH>
int max_workers_t() {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_geodesic<TW, TH, 8>, 256, 0) != hipSuccess)
        return 0;
    return ncu * (per > 0 ? per : 1);
}
}  // namespace

hipError_t launch_geodesic(const PairDev* d_pairs, const RunDev& run, int tile_w, int tile_h, int workers,
                           hipStream_t s) {
    const bool c8 = run.conn != 4;
    if (tile_w == 64 && tile_h == 16)
        return c8 ? launch_t<64, 16, 8>(d_pairs, run, workers, s) : launch_t<64, 16, 4>(d_pairs, run, workers, s);
    if (tile_w == 64 && tile_h == 32)
        return c8 ? launch_t<64, 32, 8>(d_pairs, run, workers, s) : launch_t<64, 32, 4>(d_pairs, run, workers, s);
    return c8 ? launch_t<32, 32, 8>(d_pairs, run, workers, s) : launch_t<32, 32, 4>(d_pairs, run, workers, s);
}

int geodesic_max_workers(int tile_w, int tile_h) {
    if (tile_w == 64 && tile_h == 16) return max_workers_t<64, 16>();
    if (tile_w == 64 && tile_h == 32) return max_workers_t<64, 32>();
    return max_workers_t<32, 32>();
}

}  // namespace epic
