// k_geodesic.hip -- geodesic distance transform and geodesic Voronoi labels.
//
// Computes, for every pixel p, D(p) = min over matches m of the geodesic
// distance D_G(p, p_m) of Eq. (3) and L(p) = the minimising match (lowest
// index on ties): the assignment map of Sec. 3.4 and the first term of the
// approximated distance, Eq. (4).  Eq. (3) is discretised on the 8-connected
// (or 4-connected) pixel graph; the step between adjacent pixels p, q costs
// len * (C(p) + C(q)) / 2 (trapezoid rule for the line integral of C).
//
// Algorithm: bulk-synchronous, tiled label-correcting relaxation.
//   * The image is cut into TW x TH tiles.  A tile is dirty when a pixel of
//     its 1-pixel halo (or a seed inside it) changed since its last visit.
//   * One pass is one launch over all tiles.  A dirty tile is loaded with
//     its halo into LDS, relaxed to a local fixpoint, written back, and the
//     neighbours behind every changed border are marked dirty for the next
//     pass.  Passes communicate only through memory across launches, so
//     plain cached loads and stores are coherent; no workgroup waits for
//     another.  A pass in which no border changed ends the transform: every
//     later pass exits at once.
//   * In-tile relaxation is push-based over a frontier: the first round
//     pushes from every reached pixel of the tile and halo; later rounds only
//     from pixels that improved in the previous round.  A push is a 64-bit
//     LDS atomic min of (D(p) + step, L(p)) into an in-tile neighbour.
//   * Each pixel's state is a packed (D, label) key, so relaxation is an
//     integer min: any relaxation order reaches the same fixpoint D (the
//     minimum over paths of the left-fold float sums); labels agree with the
//     lexicographic optimum except where rounded sums tie exactly.
//   * Blocks are mapped to tiles so that each XCD (blocks are dealt to the
//     8 XCDs round-robin) works on a contiguous band of tile rows; most halo
//     traffic then stays in one XCD's L2.
//   * A fixed number of passes is launched.  If the last one still changed
//     a border, a single-workgroup finisher continues the same passes until
//     the fixpoint, so the result never depends on the pass budget.
#include "epic_dev.h"

namespace epic {

namespace {

enum : int { B_L = 1, B_R = 2, B_T = 4, B_B = 8, B_TL = 16, B_TR = 32, B_BL = 64, B_BR = 128 };

template <int TW, int TH>
struct TileLds {
    static constexpr int LW = TW + 2, LH = TH + 2, NL = LW * LH;
    u64 key[NL];
    float cost[NL];
    unsigned short list[2][NL];
    u32 flag[2][NL];
    u64 dummy_key[256];     // per-thread targets of pushes that do not apply
    u32 dummy_flag[256];
    int n[2];
    int border;
};

// Visits one tile: load with halo, relax to a local fixpoint, write back.
// Returns (to every thread) the mask of borders with a changed pixel.
template <int TW, int TH, int CONN>
__device__ int visit_tile(const PairDev& P, int tx, int ty, bool first, TileLds<TW, TH>& S, int* error) {
    constexpr int NG = 256 / TW, PPT = TH / NG;
    constexpr int LW = TileLds<TW, TH>::LW, NL = TileLds<TW, TH>::NL;
    constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    static_assert(NG * TW == 256 && PPT * NG == TH, "tile shape");
    const int tid = threadIdx.x;
    const int lx = tid % TW, grp = tid / TW;
    const int x0 = tx * TW, y0 = ty * TH, W = P.W, H = P.H;
    const int twe = min(TW, W - x0), the = min(TH, H - y0);

    for (int i = tid; i < NL; i += 256) {
        const int ly = i / LW, lxx = i - ly * LW;
        const int gx = x0 + lxx - 1, gy = y0 + ly - 1;
        u64 k = KEY_INF;
        float c = 0.0f;
        if (gx >= 0 && gy >= 0 && gx < W && gy < H) {
            const long long gi = (long long)gy * W + gx;
            k = P.keys[gi];
            c = P.cost[gi];
        }
        S.key[i] = k;
        S.cost[i] = c;
        S.flag[0][i] = 0u;
        S.flag[1][i] = 0u;
    }
    if (tid == 0) {
        S.n[0] = 0;
        S.n[1] = 0;
        S.border = 0;
    }
    __syncthreads();
    u64 orig[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) orig[j] = S.key[(grp * PPT + j + 1) * LW + lx + 1];

    // Initial frontier: the reached halo pixels, and on the first pass the
    // reached pixels inside the tile (its seeds).  A tile visited before is
    // at a fixpoint relative to its previous halo, so only the halo can
    // bring anything new.
    for (int i0 = 0; i0 < NL; i0 += 256) {
        const int i = i0 + tid;
        const int iy = i / LW, ix = i - iy * LW;
        const bool halo = iy == 0 || ix == 0 || iy > the || ix > twe;
        const bool add = i < NL && key_label(S.key[i]) != NO_LABEL && (first || halo);
        const u64 mask = __ballot(add);
        if (mask) {
            const int leader = __ffsll((long long)mask) - 1;
            int base = 0;
            if ((tid & 63) == leader) base = atomicAdd(&S.n[0], __popcll(mask));
            base = __builtin_amdgcn_readlane(base, leader);
            if (add) {
                const int pos = base + (int)__builtin_amdgcn_mbcnt_hi((u32)(mask >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
                S.list[0][pos] = (unsigned short)i;
                S.flag[0][i] = 1u;
            }
        }
    }
    __syncthreads();

    int par = 0;
    const int round_cap = 4 * NL;
    for (int round = 0;; ++round) {
        const int nf = S.n[par];
        if (nf == 0) break;
        if (round > round_cap) {
            if (tid == 0) atomicOr(error, 2);
            break;
        }
        const int nxt = par ^ 1;
        for (int i0 = 0; i0 < nf; i0 += 256) {
            const int i = i0 + tid;
            const bool act = i < nf;
            int pidx = 0;
            if (act) {
                pidx = S.list[par][i];
                S.flag[par][pidx] = 0u;
            }
            const u64 kp = act ? S.key[pidx] : KEY_INF;
            const int py = pidx / LW, px = pidx - py * LW;
            const float dp = key_dist(kp);
            const u32 lp = key_label(kp);
            const float cp = S.cost[pidx];
            // The pushes are independent and branch-free: a push that does not
            // apply targets this thread's dummy slot with a key that never
            // lowers it, so the reads, atomic mins and flag claims issue as
            // three back-to-back batches of LDS operations.
            int q[CONN];
            bool ok[CONN];
#pragma unroll
            for (int k = 0; k < CONN; ++k) {
                const int qy = py + DY[k], qx = px + DX[k];
                ok[k] = act && qy >= 1 && qy <= the && qx >= 1 && qx <= twe;
                q[k] = ok[k] ? qy * LW + qx : 0;
            }
            float cq[CONN];
#pragma unroll
            for (int k = 0; k < CONN; ++k) cq[k] = S.cost[q[k]];
            u64 old[CONN], cand[CONN];
#pragma unroll
            for (int k = 0; k < CONN; ++k) {
                const float len = (k < 4) ? 1.0f : 1.41421356237309515f;
                cand[k] = ok[k] ? make_key(dp + len * (0.5f * (cp + cq[k])), lp) : ~0ull;
                old[k] = atomicMin(ok[k] ? &S.key[q[k]] : &S.dummy_key[tid], cand[k]);
            }
            u32 fo[CONN];
#pragma unroll
            for (int k = 0; k < CONN; ++k) {
                ok[k] = ok[k] && cand[k] < old[k];
                fo[k] = atomicExch(ok[k] ? &S.flag[nxt][q[k]] : &S.dummy_flag[tid], 1u);
            }
            u32 bits = 0;
#pragma unroll
            for (int k = 0; k < CONN; ++k)
                if (ok[k] && fo[k] == 0u) bits |= 1u << k;
            // append: per direction a ballot, one LDS atomic per wavefront
            u64 masks[CONN];
            int total = 0;
#pragma unroll
            for (int k = 0; k < CONN; ++k) {
                masks[k] = __ballot((bits >> k) & 1u);
                total += __popcll(masks[k]);
            }
            if (total) {
                int base = 0;
                if ((tid & 63) == 0) base = atomicAdd(&S.n[nxt], total);
                base = __builtin_amdgcn_readfirstlane(base);
#pragma unroll
                for (int k = 0; k < CONN; ++k) {
                    if ((bits >> k) & 1u) {
                        const int pos = base + (int)__builtin_amdgcn_mbcnt_hi(
                                                   (u32)(masks[k] >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((u32)masks[k], 0u));
                        S.list[nxt][pos] = (unsigned short)q[k];
                    }
                    base += __popcll(masks[k]);
                }
            }
        }
        __syncthreads();
        if (tid == 0) S.n[par] = 0;
        par = nxt;
        __syncthreads();
    }

    // write back the improved pixels and note the borders they lie on
    int bm = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ly = grp * PPT + j;
        const u64 k = S.key[(ly + 1) * LW + lx + 1];
        if (lx < twe && ly < the && k != orig[j]) {
            P.keys[(long long)(y0 + ly) * W + x0 + lx] = k;
            const bool l = lx == 0, r = lx == twe - 1, t = ly == 0, b = ly == the - 1;
            bm |= (l ? B_L : 0) | (r ? B_R : 0) | (t ? B_T : 0) | (b ? B_B : 0) | ((l && t) ? B_TL : 0) |
                  ((r && t) ? B_TR : 0) | ((l && b) ? B_BL : 0) | ((r && b) ? B_BR : 0);
        }
    }
    if (bm) atomicOr(&S.border, bm);
    __syncthreads();
    const int border = S.border;
    __syncthreads();
    return border;
}

// Marks the tiles behind changed borders dirty for pass `next`.
template <int CONN>
__device__ void mark_neighbours(const PairDev& P, const RunDev& run, int tx, int ty, int border, int next) {
    u32* dirty = run.dirty[next & 1] + P.tile_base;
    const int nx = P.tiles_x, ny = P.tiles_y;
    auto mark = [&](int cx, int cy) {
        if (cx >= 0 && cy >= 0 && cx < nx && cy < ny) dirty[cy * nx + cx] = 1u;
    };
    if (border & B_L) mark(tx - 1, ty);
    if (border & B_R) mark(tx + 1, ty);
    if (border & B_T) mark(tx, ty - 1);
    if (border & B_B) mark(tx, ty + 1);
    if (CONN == 8) {
        if (border & B_TL) mark(tx - 1, ty - 1);
        if (border & B_TR) mark(tx + 1, ty - 1);
        if (border & B_BL) mark(tx - 1, ty + 1);
        if (border & B_BR) mark(tx + 1, ty + 1);
    }
}

}  // namespace

// One pass over all tiles of all pairs.
template <int TW, int TH, int CONN>
__global__ __launch_bounds__(256) void k_geo_pass(const PairDev* __restrict__ pairs, RunDev run, int pass) {
    __shared__ TileLds<TW, TH> S;
    if (pass > 0 && run.any[pass - 1] == 0) return;          // converged
    // XCD-aware: blocks b, b+8, b+16, ... share an XCD; give each XCD a
    // contiguous run of tiles (rows of tiles are contiguous in the ids)
    const int per_xcd = (run.total_tiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (tile >= run.total_tiles) return;
    u32* dirty = run.dirty[pass & 1];
    if (dirty[tile] == 0u) return;
    const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
    const PairDev& P = pairs[p];
    const int lt = tile - P.tile_base;
    const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
    __syncthreads();
    if (threadIdx.x == 0) dirty[tile] = 0u;                  // reused two passes later
    const int border = visit_tile<TW, TH, CONN>(P, tx, ty, pass == 0, S, run.error);
    if (threadIdx.x == 0) {
        atomicAdd(&P.counters[C_TILE_VISITS], 1);
        if (border) {
            mark_neighbours<CONN>(P, run, tx, ty, border, pass + 1);
            run.any[pass] = 1;
        }
    }
}

// Continues the passes in one workgroup until no border changes (only runs
// when the launched passes did not reach the fixpoint).
template <int TW, int TH, int CONN>
__global__ __launch_bounds__(256) void k_geo_finish(const PairDev* __restrict__ pairs, RunDev run, int pass0) {
    __shared__ TileLds<TW, TH> S;
    __shared__ int s_any;
    if (run.any[pass0 - 1] == 0) return;
    for (int pass = pass0; pass < pass0 + 65536; ++pass) {
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        u32* dirty = run.dirty[pass & 1];
        for (int tile = 0; tile < run.total_tiles; ++tile) {
            if (dirty[tile] == 0u) continue;                 // uniform: same load in all threads
            const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
            const PairDev& P = pairs[p];
            const int lt = tile - P.tile_base;
            const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
            __syncthreads();
            if (threadIdx.x == 0) dirty[tile] = 0u;
            const int border = visit_tile<TW, TH, CONN>(P, tx, ty, false, S, run.error);
            if (threadIdx.x == 0) {
                atomicAdd(&P.counters[C_TILE_VISITS], 1);
                if (border) {
                    mark_neighbours<CONN>(P, run, tx, ty, border, pass + 1);
                    s_any = 1;
                }
            }
            __threadfence_block();
            __syncthreads();
        }
        __syncthreads();
        if (s_any == 0) return;
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicOr(run.error, 1);
}

namespace {
template <int TW, int TH, int CONN>
hipError_t launch_t(const PairDev* d_pairs, const RunDev& run, int passes, hipStream_t s) {
    const int grid = 8 * ((run.total_tiles + 7) / 8);
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL((k_geo_pass<TW, TH, CONN>), dim3(grid), dim3(256), 0, s, d_pairs, run, p);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_geo_finish<TW, TH, CONN>), dim3(1), dim3(256), 0, s, d_pairs, run, passes);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_geodesic(const PairDev* d_pairs, const RunDev& run, int tile_w, int tile_h, int passes,
                           hipStream_t s) {
    const bool c8 = run.conn != 4;
    if (tile_w == 64 && tile_h == 16)
        return c8 ? launch_t<64, 16, 8>(d_pairs, run, passes, s) : launch_t<64, 16, 4>(d_pairs, run, passes, s);
    if (tile_w == 64 && tile_h == 32)
        return c8 ? launch_t<64, 32, 8>(d_pairs, run, passes, s) : launch_t<64, 32, 4>(d_pairs, run, passes, s);
    return c8 ? launch_t<32, 32, 8>(d_pairs, run, passes, s) : launch_t<32, 32, 4>(d_pairs, run, passes, s);
}

}  // namespace epic
