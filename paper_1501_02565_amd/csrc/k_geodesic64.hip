// k_geodesic64.hip -- the geodesic Voronoi transform in double precision (the
// FP64-everywhere path, used for comparison with the FP32 path).
//
// Same quantity as k_geodesic.hip: D(p) = min over matches of the
// discretised geodesic distance of Eq. (3), L(p) = the minimising match,
// lowest index on ties (Sec. 3.4).  A 96-bit (D, label) pair cannot be
// relaxed with one 64-bit atomic, so the transform runs in two phases:
//   1. distances: each pixel's state is the bit pattern of a non-negative
//      double (ordered like the value), relaxed to the fixpoint -- the
//      minimum over paths of the left-fold sums D(q) + len*(C(p)+C(q))/2,
//      evaluated with explicit round-to-nearest adds and multiplies (no
//      fused multiply-add), so every sum is rounded exactly as a plain
//      double evaluation of the same expression;
//   2. labels: with D fixed, L(p) = the lowest label among the neighbours q
//      with D(q) + step(q, p) == D(p) (the predecessors on shortest
//      paths), seeds keep their own index.  Its fixpoint is the lowest
//      match index over all shortest paths, the lexicographic (D, label)
//      optimum.
// Both phases use bulk-synchronous tiled passes like k_geodesic.hip (a first
// pass over every tile with a 2-pixel margin, then dirty tiles, rounds of
// four Gauss-Seidel line sweeps in LDS, a single-workgroup finisher) on
// 32 x 16 tiles.
#include <type_traits>

#include "epic_dev.h"

namespace epic {

namespace {

constexpr int TW = 32, TH = 16;
enum : int { B_L = 1, B_R = 2, B_T = 4, B_B = 8, B_TL = 16, B_TR = 32, B_BL = 64, B_BR = 128, B_SELF = 256 };

// A region of RW x RH pixels relaxed in LDS, with a one-pixel halo.
template <int RW, int RH>
struct Lds64 {
    static constexpr int LW = RW + 2, LH = RH + 2, NL = LW * LH;
    u64 dist[NL];            // double bits
    u32 lab[NL];
    float cost[NL];
    int flag[3];             // per round (mod 3): some pixel of the tile changed
    int rowchg[LH];          // last round in which a pixel of the row changed
    int border;
};


// PHASE 0: distances; PHASE 1: labels.  The region relaxed is the tile
// widened by MX columns and MY rows on each side (0 in the normal passes;
// the first pass of each phase uses a margin, so that seeds just outside a
// tile shape it at once); only the tile itself is written back.
template <int CONN, int PHASE, int MX = 0, int MY = 0, int NT = 256>
__device__ __forceinline__ int visit64(const PairDev& P, int tx, int ty, Lds64<TW + 2 * MX, TH + 2 * MY>& S,
                                       int* error, int soft_cap = 1 << 30) {
    constexpr int RW = TW + 2 * MX, RH = TH + 2 * MY;
    using L = Lds64<RW, RH>;
    constexpr int LW = L::LW, LH = L::LH, NL = L::NL;
    constexpr int PPT = RW * RH / NT, HR = RW / PPT;       // pixels per run, row runs per row
    static_assert(PPT * NT == RW * RH && HR * PPT == RW && HR * RH == NT && (RH / PPT) * RW == NT &&
                      RH % PPT == 0, "region shape");
    constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    const int tid = threadIdx.x;
    const int x0 = tx * TW, y0 = ty * TH, W = P.W, H = P.H;
    const int rx0 = x0 - MX, ry0 = y0 - MY;                 // region origin (may be < 0)
    const int twe = min(TW, W - x0), the = min(TH, H - y0);
    // region pixels inside the image: lx in [vx0, vx1), ly in [vy0, vy1)
    const int vx0 = MX == 0 ? 0 : max(0, -rx0), vy0 = MY == 0 ? 0 : max(0, -ry0);
    const int vx1 = min(RW, W - rx0), vy1 = min(RH, H - ry0);
    // all of a thread's loads are issued before the first is stored
    constexpr int LI = (NL + NT - 1) / NT;
    u64 ld[LI];
    u32 ll[LI];
    float lc[LI];
#pragma unroll
    for (int it = 0; it < LI; ++it) {
        const int i = tid + it * NT;
        const int ly = i / LW, lxx = i - ly * LW;
        const int gx = rx0 + lxx - 1, gy = ry0 + ly - 1;
        ld[it] = DOUBLE_INF_BITS;
        ll[it] = NO_LABEL;
        lc[it] = 0.0f;
        if (i < NL && gx >= 0 && gy >= 0 && gx < W && gy < H) {
            const long long gi = (long long)gy * W + gx;
            // the tile's own pixels are written only by this visit; the
            // margin and halo belong to neighbours that may be writing them
            // (relaxed atomics: read whole, old or new)
            const bool own = gx >= x0 && gy >= y0 && gx < x0 + twe && gy < y0 + the;
            if (PHASE == 0) ld[it] = own ? gmem(P.keys)[gi] : dev_ld(P.keys + gi);
            else ld[it] = gmem(P.keys)[gi];          // distances are final in the label phase
            if (PHASE == 1) ll[it] = own ? gmem(P.labels)[gi] : dev_ld(P.labels + gi);
            lc[it] = gmem(P.cost)[gi];
        }
    }
#pragma unroll
    for (int it = 0; it < LI; ++it) {
        const int i = tid + it * NT;
        if (i < NL) {
            S.dist[i] = ld[it];
            S.lab[i] = ll[it];
            S.cost[i] = lc[it];
        }
    }
    if (tid < 3) S.flag[tid] = 0;
    for (int i = tid; i < LH; i += NT) S.rowchg[i] = -1;
    if (tid == 0) S.border = 0;
    __syncthreads();

    const int hy = tid / HR, hx = (tid % HR) * PPT;
    const int vx = tid % RW, vy = (tid / RW) * PPT;
    double wh[PPT][CONN], wv[PPT][CONN];
    u64 orig[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ch = (hy + 1) * LW + hx + j + 1, cv = (vy + j + 1) * LW + vx + 1;
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            wh[j][k] = step_f64(S.cost[ch], S.cost[ch + DY[k] * LW + DX[k]], k);
            wv[j][k] = step_f64(S.cost[cv], S.cost[cv + DY[k] * LW + DX[k]], k);
        }
        orig[j] = PHASE == 0 ? lds_ld(&S.dist[ch]) : (u64)lds_ld(&S.lab[ch]);
    }
    // every thread has its pixels' values as loaded before any sweep writes
    // (a value improved by another wave before it was read here would look
    // unchanged at write-back and never reach global memory)
    __syncthreads();
    const int round_cap = 4 * NL + 8;
    bool unconverged = false;
    for (int round = 0;; ++round) {
        int changed = 0;
        auto sweep = [&](auto rows_c, auto fwd_c) {
            constexpr bool ROWS = decltype(rows_c)::value, FWD = decltype(fwd_c)::value;
#pragma unroll
            for (int jj = 0; jj < PPT; ++jj) {
                const int j = FWD ? jj : PPT - 1 - jj;
                const int lx = ROWS ? hx + j : vx, ly = ROWS ? hy : vy + j;
                if (lx < vx0 || lx >= vx1 || ly < vy0 || ly >= vy1) continue;   // outside the image
                const int ci = (ly + 1) * LW + lx + 1;
                if (PHASE == 0) {
                    const double now = dbits(lds_ld(&S.dist[ci]));
                    double best = now;
#pragma unroll
                    for (int k = 0; k < CONN; ++k) {
                        const double cand = relax_f64(dbits(lds_ld(&S.dist[ci + DY[k] * LW + DX[k]])),
                                                      ROWS ? wh[j][k] : wv[j][k]);
                        best = cand < best ? cand : best;
                    }
                    if (best < now) {
                        lds_st(&S.dist[ci], bitsd(best));
                        lds_st(&S.rowchg[ly + 1], round);
                        changed = 1;
                    }
                } else {
                    // distances are fixed in this phase (no writer)
                    const double dp = dbits(S.dist[ci]);
                    const u32 now = lds_ld(&S.lab[ci]);
                    u32 best = now;
#pragma unroll
                    for (int k = 0; k < CONN; ++k) {
                        const int q = ci + DY[k] * LW + DX[k];
                        const bool tight = relax_f64(dbits(S.dist[q]), ROWS ? wh[j][k] : wv[j][k]) == dp;
                        const u32 lq = lds_ld(&S.lab[q]);
                        best = (tight && lq < best) ? lq : best;
                    }
                    if (best < now) {
                        lds_st(&S.lab[ci], best);
                        lds_st(&S.rowchg[ly + 1], round);
                        changed = 1;
                    }
                }
            }
        };
        // rounds of four sweeps (rows and columns, both directions) with one
        // barrier; a wavefront skips its sweeps when no pixel within one row
        // of its runs changed since the previous round started; racing
        // stores (relaxed atomics: never torn) only cost further rounds
        // (every value written is a valid distance or label, all pixels are
        // relaxed until a round changes nothing)
        bool act_h = round == 0, act_v = round == 0;
        if (round != 0) {
            act_h = max(max(lds_ld(&S.rowchg[hy]), lds_ld(&S.rowchg[hy + 1])), lds_ld(&S.rowchg[hy + 2])) >= round - 1;
            int mrow = lds_ld(&S.rowchg[vy]);
#pragma unroll
            for (int j = 1; j < PPT + 2; ++j) mrow = max(mrow, lds_ld(&S.rowchg[vy + j]));
            act_v = mrow >= round - 1;
        }
        const bool wave_h = __builtin_amdgcn_ballot_w64(act_h) != 0ull;
        const bool wave_v = __builtin_amdgcn_ballot_w64(act_v) != 0ull;
        using T = std::true_type;
        using F = std::false_type;
        if (wave_h) sweep(T{}, T{});
        if (wave_v) sweep(F{}, T{});
        if (wave_h) sweep(T{}, F{});
        if (wave_v) sweep(F{}, F{});
        if (tid == 0) lds_st(&S.flag[(round + 1) % 3], 0);
        if (__builtin_amdgcn_ballot_w64(changed != 0) != 0ull && (tid & 63) == 0) lds_st(&S.flag[round % 3], 1);
        __syncthreads();
        if (lds_ld(&S.flag[round % 3]) == 0) break;
        if (round + 1 >= soft_cap) {       // stop early; the next pass continues
            unconverged = true;
            break;
        }
        if (round > round_cap) {
            if (tid == 0) atomicOr(error, 1);     // this pair's round bound
            break;
        }
    }

    int bm = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int rlx = hx + j, rly = hy;                    // region coordinates
        const int ci = (rly + 1) * LW + rlx + 1;
        const int lx = rlx - MX, ly = rly - MY;              // tile coordinates
        const u64 v = PHASE == 0 ? S.dist[ci] : (u64)S.lab[ci];
        if (lx >= 0 && ly >= 0 && lx < twe && ly < the && v != orig[j]) {
            const long long gi = (long long)(y0 + ly) * W + x0 + lx;
            if (PHASE == 0) dev_st(P.keys + gi, v); else dev_st(P.labels + gi, (u32)v);
            const bool l = lx == 0, r = lx == twe - 1, t = ly == 0, b = ly == the - 1;
            if (MX != 0 || MY != 0 || PHASE == 1) {
                // first pass (the neighbours' values are not known yet) and
                // label phase: every neighbour behind a changed border
                bm |= (l ? B_L : 0) | (r ? B_R : 0) | (t ? B_T : 0) | (b ? B_B : 0) | ((l && t) ? B_TL : 0) |
                      ((r && t) ? B_TR : 0) | ((l && b) ? B_BL : 0) | ((r && b) ? B_BR : 0);
            } else if (l || r || t || b) {
                // distance phase: a neighbour tile only needs a visit if this
                // pixel shortens one of its pixels next to it; the halo holds
                // their distances as loaded, never lower than now
#pragma unroll
                for (int kk = 0; kk < CONN; ++kk) {
                    const int qx = lx + DX[kk], qy = ly + DY[kk];
                    const bool out = qx < 0 || qy < 0 || qx >= twe || qy >= the;
                    if (!out) continue;
                    const int qi = ci + DY[kk] * LW + DX[kk];
                    const double w = step_f64(S.cost[ci], S.cost[qi], kk);
                    if (relax_f64(dbits(v), w) < dbits(S.dist[qi])) {
                        const bool ql = qx < 0, qr = qx >= twe, qt = qy < 0, qb = qy >= the;
                        bm |= (ql && !qt && !qb) ? B_L : (qr && !qt && !qb) ? B_R
                            : (qt && !ql && !qr) ? B_T : (qb && !ql && !qr) ? B_B
                            : (ql && qt) ? B_TL : (qr && qt) ? B_TR : (ql && qb) ? B_BL : B_BR;
                    }
                }
            }
        }
    }
    if (bm) atomicOr(&S.border, bm);
    __syncthreads();
    const int border = S.border | (unconverged ? B_SELF : 0);
    __syncthreads();
    return border;
}

template <int CONN>
__device__ void mark64(const PairDev& P, const RunDev& run, int tx, int ty, int border, int next) {
    u32* dirty = run.dirty[next & 1] + P.tile_base;
    const int nx = P.tiles_x, ny = P.tiles_y;
    auto mark = [&](int cx, int cy) {
        if (cx >= 0 && cy >= 0 && cx < nx && cy < ny) dirty[cy * nx + cx] = 1u;
    };
    if (border & B_SELF) mark(tx, ty);
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

// Rounds after which a visit of a pass stops and marks its own tile for the
// next pass (values only ever decrease, so stopping early never changes the
// result; a pass no longer waits for its few slowest tiles).
constexpr int kPass64Rounds = 5;

template <int CONN, int PHASE>
__global__ __launch_bounds__(256) void k_geo64_pass(const PairDev* __restrict__ pairs, RunDev run, int pass) {
    __shared__ Lds64<TW, TH> S;
    int* any = PHASE == 0 ? run.any : run.any2;
    if (pass > 0 && any[pass - 1] == 0) return;
    // block b takes tile b: the dirty tiles, which cluster in space, are
    // spread over the XCDs (blocks are dealt to them in turn)
    const int tile = (int)blockIdx.x;
    if (tile >= run.total_tiles) return;
    u32* dirty = run.dirty[pass & 1];
    if (dirty[tile] == 0u) return;
    const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
    const PairDev& P = pairs[p];
    const int lt = tile - P.tile_base;
    const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
    __syncthreads();
    if (threadIdx.x == 0) dirty[tile] = 0u;
    const int border = visit64<CONN, PHASE>(P, tx, ty, S, P.counters + C_GEOERR, kPass64Rounds);
    if (threadIdx.x == 0) {
        atomicAdd(&P.counters[C_TILE_VISITS], 1);
        if (border) {
            mark64<CONN>(P, run, tx, ty, border, pass + 1);
            any[pass] = 1;
        }
    }
}

// The first pass of each phase: every tile, relaxed over the tile and a
// margin of kFirst64Margin pixels around it (360 threads, runs of 2
// pixels), capped at kFirst64Rounds rounds; tiles are dealt to the XCDs in
// contiguous bands, so neighbouring regions share an L2.  Visiting every
// tile also starts the label phase from all seeds at once.
constexpr int kFirst64Margin = 2, kFirst64Threads = 360, kFirst64Rounds = 4;

template <int CONN, int PHASE>
__global__ __launch_bounds__(kFirst64Threads) void k_geo64_first(const PairDev* __restrict__ pairs, RunDev run) {
    __shared__ Lds64<TW + 2 * kFirst64Margin, TH + 2 * kFirst64Margin> S;
    int* any = PHASE == 0 ? run.any : run.any2;
    const int per_xcd = (run.total_tiles + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (tile >= run.total_tiles) return;
    const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
    const PairDev& P = pairs[p];
    const int lt = tile - P.tile_base;
    const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
    if (threadIdx.x == 0) run.dirty[0][tile] = 0u;       // this pass visits every tile
    const int border = visit64<CONN, PHASE, kFirst64Margin, kFirst64Margin, kFirst64Threads>(
        P, tx, ty, S, P.counters + C_GEOERR, kFirst64Rounds);
    if (threadIdx.x == 0) {
        atomicAdd(&P.counters[C_TILE_VISITS], 1);
        if (border) {
            mark64<CONN>(P, run, tx, ty, border, 1);
            any[0] = 1;
        }
    }
}

template <int CONN, int PHASE>
__global__ __launch_bounds__(256) void k_geo64_finish(const PairDev* __restrict__ pairs, RunDev run, int pass0) {
    __shared__ Lds64<TW, TH> S;
    __shared__ int s_any;
    int* any = PHASE == 0 ? run.any : run.any2;
    // passes that changed something (a prefix): the phase needs one more,
    // which is reported for the automatic budget of later calls
    int changed = 0;
    for (int q = 0; q < pass0; ++q) changed += any[q] != 0 ? 1 : 0;
    if (any[pass0 - 1] == 0) {
        if (threadIdx.x == 0 && run.passes_used) run.passes_used[PHASE] = changed + 1;
        return;
    }
    __shared__ int s_list[256];
    __shared__ int s_cnt;
    for (int pass = pass0; pass < pass0 + 65536; ++pass) {
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        u32* dirty = run.dirty[pass & 1];
        // dirty flags read 256 at a time in parallel, dirty tiles listed
        for (int t0 = 0; t0 < run.total_tiles; t0 += 256) {
            if (threadIdx.x == 0) s_cnt = 0;
            __syncthreads();
            const int tt = t0 + (int)threadIdx.x;
            if (tt < run.total_tiles && dirty[tt] != 0u) s_list[atomicAdd(&s_cnt, 1)] = tt;
            __syncthreads();
            const int cnt = s_cnt;
            for (int q = 0; q < cnt; ++q) {
            const int tile = s_list[q];
            const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
            const PairDev& P = pairs[p];
            const int lt = tile - P.tile_base;
            const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
            __syncthreads();
            if (threadIdx.x == 0) dirty[tile] = 0u;
            const int border = visit64<CONN, PHASE>(P, tx, ty, S, P.counters + C_GEOERR);
            if (threadIdx.x == 0) {
                atomicAdd(&P.counters[C_TILE_VISITS], 1);
                if (border) {
                    mark64<CONN>(P, run, tx, ty, border, pass + 1);
                    s_any = 1;
                }
            }
            __threadfence_block();
            __syncthreads();
            }
            __syncthreads();
        }
        __syncthreads();
        if (s_any == 0) {
            if (threadIdx.x == 0 && run.passes_used) run.passes_used[PHASE] = changed + 1;
            return;
        }
        ++changed;
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicOr(run.error, 1);
}

// Between the phases: clears the dirty flags the distance phase left.
__global__ __launch_bounds__(256) void k_geo64_reset(RunDev run) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < run.total_tiles; i += gridDim.x * 256) {
        run.dirty[0][i] = 0u;
        run.dirty[1][i] = 0u;
    }
}

namespace {
template <int CONN>
hipError_t launch64_t(const PairDev* d_pairs, const RunDev& run, int passes0, int passes1, hipStream_t s) {
    const int grid = 8 * ((run.total_tiles + 7) / 8);
    hipLaunchKernelGGL((k_geo64_first<CONN, 0>), dim3(grid), dim3(kFirst64Threads), 0, s, d_pairs, run);
    for (int p = 1; p < passes0; ++p)
        hipLaunchKernelGGL((k_geo64_pass<CONN, 0>), dim3(grid), dim3(256), 0, s, d_pairs, run, p);
    hipLaunchKernelGGL((k_geo64_finish<CONN, 0>), dim3(1), dim3(256), 0, s, d_pairs, run, passes0);
    hipLaunchKernelGGL(k_geo64_reset, dim3((run.total_tiles + 255) / 256), dim3(256), 0, s, run);
    hipLaunchKernelGGL((k_geo64_first<CONN, 1>), dim3(grid), dim3(kFirst64Threads), 0, s, d_pairs, run);
    for (int p = 1; p < passes1; ++p)
        hipLaunchKernelGGL((k_geo64_pass<CONN, 1>), dim3(grid), dim3(256), 0, s, d_pairs, run, p);
    hipLaunchKernelGGL((k_geo64_finish<CONN, 1>), dim3(1), dim3(256), 0, s, d_pairs, run, passes1);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_geodesic64(const PairDev* d_pairs, const RunDev& run, int passes0, int passes1, hipStream_t s) {
    return run.conn == 4 ? launch64_t<4>(d_pairs, run, passes0, passes1, s)
                         : launch64_t<8>(d_pairs, run, passes0, passes1, s);
}

}  // namespace epic
