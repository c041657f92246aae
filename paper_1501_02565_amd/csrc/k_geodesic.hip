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
//   * One pass is one launch.  The first visits every tile; each later one
//     walks the list of tiles marked dirty by the pass before.  A dirty tile is loaded with
//     its halo into LDS, relaxed to a local fixpoint (or for a capped number
//     of rounds, after which it marks itself dirty), written back, and the
//     neighbours behind every changed border are marked dirty for the next
//     pass.  Within a launch, a tile's halo may be read while its owner
//     writes it: those keys are read and written with relaxed atomics at
//     agent scope, so a reader gets the old or the new key whole (either
//     is a valid upper bound, and any change it misses marks it dirty for
//     the next pass).  Passes see each other's writes across launches; no
//     workgroup waits for another.  A pass in which no border changed ends the transform: every
//     later pass exits at once.
//   * In-tile relaxation is Gauss-Seidel over lines of pixels owned by one
//     thread, alternating between rows and columns and between sweep
//     directions, until a round changes nothing.
//   * Each pixel's state is a packed (D, label) key, so relaxation is an
//     integer min: any relaxation order reaches the same fixpoint D (the
//     minimum over paths of the left-fold float sums); labels agree with the
//     lexicographic optimum except where rounded sums tie exactly.
//   * In the first pass (every tile busy) blocks are mapped to tiles so that
//     each XCD (blocks are dealt to the 8 XCDs round-robin) works on a
//     contiguous band of tile rows, keeping most halo traffic in one XCD's
//     L2; the later passes take their tiles in list order, which spreads
//     the spatially clustered dirty tiles over all XCDs.
//   * A fixed number of passes is launched.  If the last one still changed
//     a border, a single-workgroup finisher continues the same passes until
//     the fixpoint, so the result never depends on the pass budget.
#include <algorithm>
#include <type_traits>

#include "epic_dev.h"

namespace epic {

namespace {

// Minimum of two doubles as one v_min_f64.  The operands are packed keys
// (never NaN patterns), so the IEEE-mode canonicalisation the compiler would
// insert before a minnum is not needed.
__device__ __forceinline__ double min_f64(double a, double b) {
    double r;
    __asm__("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Minimum of the first n (compile-time after unrolling) of c[] as a
// balanced tree of min_f64.
template <int N>
__device__ __forceinline__ double tree_min(double (&c)[N], int n) {
#pragma unroll
    for (int w = 1; w < N; w <<= 1)
#pragma unroll
        for (int i = 0; i + w < N; i += 2 * w)
            if (i + w < n) c[i] = min_f64(c[i], c[i + w]);
    return c[0];
}

enum : int { B_L = 1, B_R = 2, B_T = 4, B_B = 8, B_TL = 16, B_TR = 32, B_BL = 64, B_BR = 128, B_SELF = 256,
             B_REACHED = 512 };

template <int TW, int TH>
struct TileLds {
    static constexpr int LW = TW + 2, LH = TH + 2, NL = LW * LH;
    u64 key[NL];
    float cost[NL];
    int flag[3];             // per round (mod 3): some pixel of the tile changed
    int rowchg[LH];          // last round in which a pixel of the row changed
    int border;
};

// The same with a per-pixel bound on the distances worth keeping (the exact
// interpolation's single-source transforms).
template <int TW, int TH>
struct TileLdsB : TileLds<TW, TH> {
    float ub[TileLds<TW, TH>::NL];
};
template <int TW, int TH, bool BOUND>
using TileLdsT = typename std::conditional<BOUND, TileLdsB<TW, TH>, TileLds<TW, TH>>::type;

template <class L>
__device__ __forceinline__ float bound_at(const L& S, int i) {
    if constexpr (std::is_same<L, TileLdsB<L::LW - 2, L::LH - 2>>::value) return S.ub[i];
    else return INFINITY;
}

// Visits one tile: load with halo, relax to a local fixpoint, write back.
// Returns (to every thread) the mask of borders with a changed pixel.
//
// In-tile relaxation is Gauss-Seidel over lines: each of the NT threads owns
// a run of PPT consecutive pixels along a row and one along a column.  A
// round sweeps the row run forwards, the column run forwards, the row run
// backwards and the column run backwards, updating every pixel in place from
// its 8 (or 4) neighbours; the workgroup only meets at the end of a round.
// A sweep keeps the 3 x 3 window around the current pixel in registers and
// slides it: each step reads only the three keys ahead (issued before the
// current pixel is computed), and the pixel behind is the value just
// computed.  Wavefronts may be in different sweeps at once, so a pixel's
// row-run and column-run owners can race on it, and window values may be a
// few steps old.  Every written value is the length of a real path and every
// pixel is relaxed in every round, so a lost or late update only costs
// another round: a round in which no pixel improved leaves every pixel at
// the minimum over its neighbours, which is the fixpoint.  A wavefront whose
// runs saw no change within one row since the previous round started skips
// its sweeps (per-row change rounds in LDS).  Keys and flags that several
// waves touch at once are read and written with relaxed atomics, which on
// gfx950 are the plain 64-bit LDS accesses: a key is never seen half-written.
//
// A key (D bits, label) with D >= 0 read as an IEEE double is a non-negative
// value below the NaN range whose order is the unsigned order of the key
// (denormals are kept for doubles in these kernels), so the lexicographic
// minimum over the neighbours is a chain of double minima.
// Index k of the neighbour at (dx, dy) in DX/DY order, or -1.
constexpr int nb_index(int dx, int dy) {
    return dx == 1 && dy == 0 ? 0 : dx == -1 && dy == 0 ? 1 : dx == 0 && dy == 1 ? 2 : dx == 0 && dy == -1 ? 3
         : dx == 1 && dy == 1 ? 4 : dx == -1 && dy == 1 ? 5 : dx == 1 && dy == -1 ? 6 : dx == -1 && dy == -1 ? 7 : -1;
}

//
// The region relaxed is the tile widened by MX columns and MY rows on each
// side (both 0 in the normal passes); only the tile itself is written back.
// The first pass uses a margin so that seeds just outside a tile already
// shape its distances, which saves most of the passes that would otherwise
// carry them in one tile at a time.
//
// BOUND: a key whose distance exceeds the pixel's bound (P.ubound, at least
// the distance of the pixel's K-th nearest match) is not taken, so a
// single-source transform only spreads where its distances can matter.  If
// the source is one of p's K nearest, every pixel q on a shortest path from
// it to p has it among its own K nearest (a match closer to q would be
// closer to p), so its distance at q is within q's bound and the path to p
// is never cut.
template <int TW, int TH, int MX, int MY, int CONN, int NT, bool BOUND = false>
__device__ __forceinline__ int visit_tile(const PairDev& P, int tx, int ty,
                                          TileLdsT<TW + 2 * MX, TH + 2 * MY, BOUND>& S, int* error,
                                          int soft_cap = 1 << 30) {
    constexpr int RW = TW + 2 * MX, RH = TH + 2 * MY;     // region relaxed
    constexpr int PPT = RW * RH / NT;
    constexpr int LW = TileLds<RW, RH>::LW, LH = TileLds<RW, RH>::LH, NL = TileLds<RW, RH>::NL;
    constexpr int HR = RW / PPT;           // row runs per row
    static_assert(PPT * NT == RW * RH && HR * PPT == RW && HR * RH == NT && (RH / PPT) * RW == NT &&
                      RH % PPT == 0, "tile shape");
    constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    const int tid = threadIdx.x;
    const int x0 = tx * TW, y0 = ty * TH, W = P.W, H = P.H;
    const int rx0 = x0 - MX, ry0 = y0 - MY;               // region origin (may be < 0)
    const int twe = min(TW, W - x0), the = min(TH, H - y0);
    // region pixels inside the image: lx in [vx0, vx1), ly in [vy0, vy1)
    const int vx0 = MX == 0 ? 0 : max(0, -rx0), vy0 = MY == 0 ? 0 : max(0, -ry0);
    const int vx1 = min(RW, W - rx0), vy1 = min(RH, H - ry0);

    // all of a thread's loads are issued before the first is stored, so the
    // tile costs one memory round trip, not one per element
    constexpr int LI = (NL + NT - 1) / NT;
    u64 lk[LI];
    float lc[LI];
    float lu[BOUND ? LI : 1];
#pragma unroll
    for (int it = 0; it < LI; ++it) {
        const int i = tid + it * NT;
        const int ly = i / LW, lxx = i - ly * LW;
        const int gx = rx0 + lxx - 1, gy = ry0 + ly - 1;
        lk[it] = KEY_INF;
        lc[it] = 0.0f;
        if constexpr (BOUND) lu[it] = 0.0f;
        if (i < NL && gx >= 0 && gy >= 0 && gx < W && gy < H) {
            const long long gi = (long long)gy * W + gx;
            // the tile's own pixels are written only by this visit; the
            // margin and halo belong to neighbours that may be writing them
            const bool own = gx >= x0 && gy >= y0 && gx < x0 + twe && gy < y0 + the;
            lk[it] = own ? gmem(P.keys)[gi] : dev_ld(P.keys + gi);
            lc[it] = gmem(P.cost)[gi];
            if constexpr (BOUND) lu[it] = gmem(P.ubound)[gi];
        }
    }
#pragma unroll
    for (int it = 0; it < LI; ++it) {
        const int i = tid + it * NT;
        if (i < NL) {
            S.key[i] = lk[it];
            S.cost[i] = lc[it];
            if constexpr (BOUND) S.ub[i] = lu[it];
        }
    }
    if (tid < 3) S.flag[tid] = 0;
    for (int i = tid; i < LH; i += NT) S.rowchg[i] = -1;
    if (tid == 0) S.border = 0;
    __syncthreads();

    // the two runs of this thread: a row run (hx.., hy) and a column run
    // (vx, vy..), with their step costs to the 8 neighbours
    const int hy = tid / HR, hx = (tid % HR) * PPT;
    const int vx = tid % RW, vy = (tid / RW) * PPT;
    float wh[PPT][CONN], wv[PPT][CONN];
    u64 orig[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int ch = (hy + 1) * LW + hx + j + 1, cv = (vy + j + 1) * LW + vx + 1;
        const float cph = S.cost[ch], cpv = S.cost[cv];
#pragma unroll
        for (int k = 0; k < CONN; ++k) {
            const float len = (k < 4) ? 1.0f : 1.41421356237309515f;
            wh[j][k] = step_f32(len, cph, S.cost[ch + DY[k] * LW + DX[k]]);
            wv[j][k] = step_f32(len, cpv, S.cost[cv + DY[k] * LW + DX[k]]);
        }
        orig[j] = lds_ld(&S.key[ch]);
    }
    // every thread has its pixels' values as loaded before any sweep writes
    // (a value improved by another wave before it was read here would look
    // unchanged at write-back and never reach global memory)
    __syncthreads();
    const int round_cap = 4 * NL + 8;
    bool unconverged = false;
    for (int round = 0;; ++round) {
        int changed = 0;
        // one sweep of one of this thread's runs; ROWS and FWD are
        // compile-time so the step-cost registers are indexed statically
        auto sweep = [&](auto rows_c, auto fwd_c) {
            constexpr bool ROWS = decltype(rows_c)::value, FWD = decltype(fwd_c)::value;
            constexpr int SA = (FWD ? 1 : -1) * (ROWS ? 1 : LW);   // one step along the run
            constexpr int SB = ROWS ? LW : 1;                     // one step across it
            const int j0 = FWD ? 0 : PPT - 1;
            int c = ROWS ? (hy + 1) * LW + hx + j0 + 1 : (vy + j0 + 1) * LW + vx + 1;
            // win[a + 1][b + 1]: the key a steps along and b steps across
            u64 win[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) win[a][b] = lds_ld(&S.key[c + (a - 1) * SA + (b - 1) * SB]);
#pragma unroll
            for (int jj = 0; jj < PPT; ++jj) {
                const int j = FWD ? jj : PPT - 1 - jj;
                u64 nxt[3] = {0, 0, 0};
                if (jj + 1 < PPT) {
#pragma unroll
                    for (int b = 0; b < 3; ++b) nxt[b] = lds_ld(&S.key[c + 2 * SA + (b - 1) * SB]);
                }
                const int lx = ROWS ? hx + j : vx, ly = ROWS ? hy : vy + j;
                const u64 now = win[1][1];
                // candidates from keys read from LDS are reduced as a tree;
                // the one from the pixel just computed (behind, jj > 0) is
                // taken last, so consecutive pixels overlap
                constexpr int NC = CONN + 1;
                double cand[NC];
                int nc = 0;
                cand[nc++] = __longlong_as_double((long long)now);
                double behind = cand[0];
#pragma unroll
                for (int a = -1; a <= 1; ++a) {
#pragma unroll
                    for (int b = -1; b <= 1; ++b) {
                        const int al = FWD ? a : -a;           // along, in +x / +y terms
                        const int k = ROWS ? nb_index(al, b) : nb_index(b, al);
                        if (k < 0 || k >= CONN) continue;
                        const u64 q = win[a + 1][b + 1];
                        const float w = ROWS ? wh[j][k] : wv[j][k];
                        const double cd = __longlong_as_double((long long)make_key(relax_f32(key_dist(q), w), key_label(q)));
                        if (a == -1 && b == 0 && jj > 0) behind = cd; else cand[nc++] = cd;
                    }
                }
                double best = tree_min<NC>(cand, nc);
                if (jj > 0) best = min_f64(best, behind);
                u64 bk = (u64)__double_as_longlong(best);
                if (lx < vx0 || lx >= vx1 || ly < vy0 || ly >= vy1) bk = now;   // outside the image
                if constexpr (BOUND) {
                    if (key_dist(bk) > S.ub[c]) bk = now;                    // beyond the bound
                }
                if (bk < now) {
                    lds_st(&S.key[c], bk);
                    lds_st(&S.rowchg[ly + 1], round);
                    changed = 1;
                }
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    win[0][b] = win[1][b];
                    win[1][b] = win[2][b];
                    win[2][b] = nxt[b];
                }
                win[0][1] = bk;
                c += SA;
            }
        };
        using T = std::true_type;
        using F = std::false_type;
        // a wavefront skips its row (column) sweeps when no pixel within
        // one row of its runs changed since the start of the previous round:
        // then none of its pixels can improve
        bool act_h = round == 0, act_v = round == 0;
        if (round != 0) {
            act_h = max(max(lds_ld(&S.rowchg[hy]), lds_ld(&S.rowchg[hy + 1])), lds_ld(&S.rowchg[hy + 2])) >= round - 1;
            int m = lds_ld(&S.rowchg[vy]);
#pragma unroll
            for (int j = 1; j < PPT + 2; ++j) m = max(m, lds_ld(&S.rowchg[vy + j]));
            act_v = m >= round - 1;
        }
        const bool wave_h = __builtin_amdgcn_ballot_w64(act_h) != 0ull;
        const bool wave_v = __builtin_amdgcn_ballot_w64(act_v) != 0ull;
        if (wave_h) sweep(T{}, T{});
        if (wave_v) sweep(F{}, T{});
        if (wave_h) sweep(T{}, F{});
        if (wave_v) sweep(F{}, F{});
        // flag this round's changes per wavefront (the flag of the next
        // round was last read two rounds ago) and meet
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

    // write back the improved pixels and note the borders they lie on
    int bm = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int lx = hx + j - MX, ly = hy - MY;          // tile coordinates
        const u64 k = S.key[(hy + 1) * LW + hx + j + 1];
        if constexpr (BOUND) {
            if (lx >= 0 && ly >= 0 && lx < twe && ly < the && key_dist(k) < __int_as_float(0x7f800000))
                bm |= B_REACHED;
        }
        // the first pass of a bounded transform visits only the seed's tile,
        // so every reached pixel on its border must mark the tile behind it,
        // the seed itself included (the seeding wrote it, so it never
        // changes here)
        const bool spread = BOUND && (MX != 0 || MY != 0) && key_dist(k) < __int_as_float(0x7f800000);
        if (lx >= 0 && ly >= 0 && lx < twe && ly < the && (k != orig[j] || spread)) {
            if (k != orig[j]) dev_st(P.keys + (long long)(y0 + ly) * W + x0 + lx, k);
            const bool l = lx == 0, r = lx == twe - 1, t = ly == 0, b = ly == the - 1;
            if (MX != 0 || MY != 0) {
                // first pass: the neighbours' values are not known yet
                bm |= (l ? B_L : 0) | (r ? B_R : 0) | (t ? B_T : 0) | (b ? B_B : 0) | ((l && t) ? B_TL : 0) |
                      ((r && t) ? B_TR : 0) | ((l && b) ? B_BL : 0) | ((r && b) ? B_BR : 0);
            } else if (l || r || t || b) {
                // a neighbour tile only needs a visit if this pixel improves
                // one of its pixels next to it; the halo holds their values
                // as loaded (never lower than now), so the test never misses
                const int ci = (hy + 1) * LW + hx + j + 1;
                const float dp = key_dist(k), cp = S.cost[ci];
#pragma unroll
                for (int kk = 0; kk < CONN; ++kk) {
                    const int qx = lx + DX[kk], qy = ly + DY[kk];
                    const bool out = qx < 0 || qy < 0 || qx >= twe || qy >= the;
                    if (!out) continue;
                    const int qi = ci + DY[kk] * LW + DX[kk];
                    const float len = (kk < 4) ? 1.0f : 1.41421356237309515f;
                    // priced exactly as the neighbour's sweep would price it
                    const u64 cand = make_key(relax_f32(dp, step_f32(len, cp, S.cost[qi])), key_label(k));
                    if (cand < S.key[qi] && (!BOUND || key_dist(cand) <= bound_at(S, qi))) {
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
    int border = S.border | (unconverged ? B_SELF : 0);
    __syncthreads();
    if constexpr (BOUND) {
        // the box of tiles this pair's distances reached
        if ((border & B_REACHED) && tid == 0) {
            atomicMax(&P.counters[C_BX0], (1 << 24) - tx);
            atomicMax(&P.counters[C_BY0], (1 << 24) - ty);
            atomicMax(&P.counters[C_BX1], 1 + tx);
            atomicMax(&P.counters[C_BY1], 1 + ty);
        }
        border &= ~B_REACHED;
    }
    return border;
}

// Marks the tiles behind changed borders dirty for pass `next`; called by
// every thread of the workgroup with the (uniform) border mask.  With
// LISTED, thread k < 9 takes direction k (its exchange and append round
// trips overlap the others'), and a tile whose flag it sets is appended to
// the pass's dirty-tile list (the exchange lets each tile enter once);
// without, thread 0 stores the flags (passes that visit every flagged tile
// by scanning).
template <int CONN, bool LISTED>
__device__ void mark_neighbours(const PairDev& P, const RunDev& run, int tx, int ty, int border, int next) {
    constexpr int BIT[9] = {B_SELF, B_L, B_R, B_T, B_B, B_TL, B_TR, B_BL, B_BR};
    constexpr int DXK[9] = {0, -1, 1, 0, 0, -1, 1, -1, 1};
    constexpr int DYK[9] = {0, 0, 0, -1, 1, -1, -1, 1, 1};
    constexpr int ND = CONN == 8 ? 9 : 5;
    if (!LISTED) {
        // plain stores, issued one after another by one thread (measured
        // faster than spreading them over lanes)
        if (threadIdx.x != 0) return;
        EPIC_GLOBAL u32* dirty = gmem(run.dirty[next & 1]) + P.tile_base;
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            const int cx = tx + DXK[k], cy = ty + DYK[k];
            if ((border & BIT[k]) && cx >= 0 && cy >= 0 && cx < P.tiles_x && cy < P.tiles_y)
                dirty[cy * P.tiles_x + cx] = 1u;
        }
        return;
    }
    const int k = threadIdx.x;
    if (k >= ND || !(border & BIT[k])) return;
    const int cx = tx + DXK[k], cy = ty + DYK[k];
    if (cx < 0 || cy < 0 || cx >= P.tiles_x || cy >= P.tiles_y) return;
    const int t = cy * P.tiles_x + cx;
    if (atomicExch(&run.dirty[next & 1][P.tile_base + t], 1u) == 0u) {
        const int L = next % 3;
        run.wl[L][atomicAdd(&run.wl_cnt[L], 1)] = (u32)(P.tile_base + t);
    }
}

}  // namespace

// Rounds after which a visit stops and marks its own tile for the next pass,
// which continues from the values written (every written value is the
// length of a real path, so stopping early never changes the result).  A
// pass lasts as long as its slowest visit; a few tiles need many more rounds
// than the rest, so capping them and letting the next pass (which sees the
// neighbours' newer values) finish them shortens the transform.  Measured on
// 1024x436 with 8000 matches: first pass capped at 4, later ones at 5.
constexpr int kFirstRounds = 4;
constexpr int kPassRounds = 5;

// One pass.  LISTED: the grid walks the pass's list of dirty tiles (written
// by the previous pass), so a launch costs what its dirty tiles cost however
// many tiles the pairs of the call have; the list of pass p + 2 (read by
// pass p - 1) is emptied here for pass p + 1 to fill, and list order (the
// order of marking) spreads the spatially clustered dirty tiles over the
// XCDs.  Otherwise block b takes tile b (consecutive tiles go to different
// XCDs) and returns at once when its flag is clear: cheaper for a single
// image, whose marks then are plain stores.
template <int TW, int TH, int CONN, int NT, bool LISTED, bool BOUND = false>
__global__ __launch_bounds__(NT) void k_geo_pass(const PairDev* __restrict__ pairs, RunDev run, int pass) {
    __shared__ TileLdsT<TW, TH, BOUND> S;
    // A listed pass reads its list only while the transform still changes.
    // A block-per-tile pass needs no such gate in front of its own flag (one
    // memory round trip less on every visit): every mark sets its pass's
    // change flag, and the seeding's marks are cleared by the first pass,
    // which visits every tile they name, so after a pass without changes no
    // tile of the next one is marked.
    if (LISTED && pass > 0 && run.any[pass - 1] == 0) return;
    u32* dirty = run.dirty[pass & 1];
    auto visit = [&](int tile) {
        const int p = find_pair(run.npairs, tile, [&](int k) { return pairs[k].tile_base; });
        const PairDev& P = pairs[p];
        const int lt = tile - P.tile_base;
        const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
        __syncthreads();                                     // the previous tile's LDS is done
        if (threadIdx.x == 0) dirty[tile] = 0u;              // reused two passes later
        const int border = visit_tile<TW, TH, 0, 0, CONN, NT, BOUND>(P, tx, ty, S, P.counters + C_GEOERR,
                                                                     kPassRounds);
        if (threadIdx.x == 0) atomicAdd(&P.counters[C_TILE_VISITS], 1);
        if (threadIdx.x == 0 && run.pass_visits) atomicAdd(&run.pass_visits[pass], 1);
        if (border) {
            mark_neighbours<CONN, LISTED>(P, run, tx, ty, border, pass + 1);
            if (threadIdx.x == 0) run.any[pass] = 1;
        }
    };
    if constexpr (LISTED) {
        const int cnt = run.wl_cnt[pass % 3];
        if (blockIdx.x == 0 && threadIdx.x == 0) run.wl_cnt[(pass + 2) % 3] = 0;
        const u32* list = run.wl[pass % 3];
        for (int i = (int)blockIdx.x; i < cnt; i += (int)gridDim.x) visit((int)list[i]);
    } else {
        // the flag is read before the bound is tested (its argument loads
        // then go out together): the grid is the tile count rounded up to a
        // multiple of 8 and each flag array is carved to a multiple of 64
        // entries, so the read stays within the array
        const int tile = (int)blockIdx.x;
        u32* const d0 = run.dirty[0];
        u32* const d1 = run.dirty[1];
        const u32 dflag = ((pass & 1) ? d1 : d0)[tile];
        if (tile >= run.total_tiles || dflag == 0u) return;
        visit(tile);
    }
}


// The first pass: every tile, relaxed over the tile and a margin of MX
// columns and MY rows around it (seeds from the start, written by k_seed).
// Bounded (single-source) transforms launch one block per pair instead,
// which visits the tiles holding the pair's seeds; the others are reached
// through the marks of later passes.
template <int TW, int TH, int MX, int MY, int CONN, int NT, bool LISTED, bool BOUND = false>
__global__ __launch_bounds__(NT) void k_geo_first(const PairDev* __restrict__ pairs, RunDev run) {
    __shared__ TileLdsT<TW + 2 * MX, TH + 2 * MY, BOUND> S;
    if constexpr (BOUND) {
        const PairDev& P = pairs[blockIdx.x];
        for (int m = 0; m < P.N; ++m) {
            const int sp = P.seed_pix[m];
            if (sp < 0) continue;
            const int tile = P.tile_base + (sp / P.W / TH) * P.tiles_x + (sp % P.W) / TW;
            __syncthreads();                                     // the previous visit is done
            if (run.dirty[0][tile] == 0u) continue;              // (uniform) visited already
            __syncthreads();                                     // every thread has read the flag
            const int lt = tile - P.tile_base;
            const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
            if (threadIdx.x == 0) run.dirty[0][tile] = 0u;
            const int border = visit_tile<TW, TH, MX, MY, CONN, NT, BOUND>(P, tx, ty, S, P.counters + C_GEOERR,
                                                                           kFirstRounds);
            if (threadIdx.x == 0) atomicAdd(&P.counters[C_TILE_VISITS], 1);
            if (threadIdx.x == 0 && run.pass_visits) atomicAdd(&run.pass_visits[0], 1);
            if (border) {
                mark_neighbours<CONN, LISTED>(P, run, tx, ty, border, 1);
                if (threadIdx.x == 0) run.any[0] = 1;
            }
        }
        return;
    } else {
        const int per_xcd = (run.total_tiles + 7) / 8;
        const int tile = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
        if (tile >= run.total_tiles) return;
        const int p = find_pair(run.npairs, tile, [&](int i) { return pairs[i].tile_base; });
        const PairDev& P = pairs[p];
        const int lt = tile - P.tile_base;
        const int tx = lt % P.tiles_x, ty = lt / P.tiles_x;
        if (threadIdx.x == 0) run.dirty[0][tile] = 0u;           // reused by pass 2
        const int border = visit_tile<TW, TH, MX, MY, CONN, NT, BOUND>(P, tx, ty, S, P.counters + C_GEOERR,
                                                                       kFirstRounds);
        if (threadIdx.x == 0) atomicAdd(&P.counters[C_TILE_VISITS], 1);
        if (threadIdx.x == 0 && run.pass_visits) atomicAdd(&run.pass_visits[0], 1);
        if (border) {
            mark_neighbours<CONN, LISTED>(P, run, tx, ty, border, 1);
            if (threadIdx.x == 0) run.any[0] = 1;
        }
    }
}

// Continues the passes in one workgroup until no border changes (only runs
// when the launched passes did not reach the fixpoint).
template <int TW, int TH, int CONN, int NT, bool BOUND = false>
__global__ __launch_bounds__(NT) void k_geo_finish(const PairDev* __restrict__ pairs, RunDev run, int pass0) {
    __shared__ TileLdsT<TW, TH, BOUND> S;
    __shared__ int s_any;
    // passes that changed something so far (they form a prefix): the
    // transform needs one more than that, which is reported for the
    // automatic pass budget of later calls
    int changed = 0;
    for (int q = 0; q < pass0; ++q) changed += run.any[q] != 0 ? 1 : 0;
    if (run.any[pass0 - 1] == 0) {
        if (threadIdx.x == 0 && run.passes_used) *run.passes_used = changed + 1;
        return;
    }
    __shared__ int s_list[NT];
    __shared__ int s_cnt;
    for (int pass = pass0; pass < pass0 + 65536; ++pass) {
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        u32* dirty = run.dirty[pass & 1];
        // the dirty flags of NT tiles at a time are read in parallel and the
        // dirty tiles listed (a batch of a million tiles is mostly clean);
        // tiles are visited in any order, the fixpoint being unique
        for (int t0 = 0; t0 < run.total_tiles; t0 += NT) {
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
            const int border = visit_tile<TW, TH, 0, 0, CONN, NT, BOUND>(P, tx, ty, S, P.counters + C_GEOERR);
            if (threadIdx.x == 0) atomicAdd(&P.counters[C_TILE_VISITS], 1);
            if (threadIdx.x == 0 && run.pass_visits) atomicAdd(&run.pass_visits[min(pass, kMaxPasses - 1)], 1);
            if (border) {
                mark_neighbours<CONN, false>(P, run, tx, ty, border, pass + 1);
                if (threadIdx.x == 0) s_any = 1;
            }
            __threadfence_block();
            __syncthreads();
            }
            __syncthreads();
        }
        __syncthreads();
        if (s_any == 0) {
            if (threadIdx.x == 0 && run.passes_used) *run.passes_used = changed + 1;
            return;
        }
        ++changed;
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicOr(run.error, 1);
}

namespace {
// First-pass margin (pixels on each side) and threads: a 32 x 16 tile
// becomes a 36 x 20 region relaxed by 180 threads (runs of 4 pixels), 32 x 32
// a 40 x 40 region (800 threads, runs of 2), 32 x 64 a 40 x 72 region (720
// threads, runs of 4).  Margins of 2 to 4 measured alike on 32 x 16 tiles;
// wider ones make the first pass the longest.  Runs of 4 take as long as
// runs of 2 on one pair with half the wavefronts, which helps batches.
constexpr int first_margin(int th) { return th == 16 ? 2 : 4; }
constexpr int first_threads(int th) { return th == 16 ? 180 : th == 32 ? 800 : 720; }

// Calls with more tiles than kListTiles walk dirty-tile lists in their
// later passes, with grids of at most kPassGrid blocks (a longer list is
// walked in turns); smaller ones launch a block per tile.  On the 64-pair
// batch (36.6k tiles) grids of 1024 and 8192 blocks measured 2 % faster than
// 2048 or 4096, and 512 7 % slower.
constexpr int kListTiles = 4096;
constexpr int kPassGrid = 1024;

template <int TW, int TH, int CONN, int NT, bool LISTED, bool BOUND = false>
hipError_t launch_l(const PairDev* d_pairs, const RunDev& run, int passes, hipStream_t s) {
    const int grid = 8 * ((run.total_tiles + 7) / 8);
    const int pgrid = LISTED ? std::min(run.total_tiles, kPassGrid) : grid;
    constexpr int NT0 = first_threads(TH), M0 = first_margin(TH);
    hipLaunchKernelGGL((k_geo_first<TW, TH, M0, M0, CONN, NT0, LISTED, BOUND>), dim3(BOUND ? run.npairs : grid),
                       dim3(NT0), 0, s, d_pairs, run);
    for (int p = 1; p < passes; ++p) {
        hipLaunchKernelGGL((k_geo_pass<TW, TH, CONN, NT, LISTED, BOUND>), dim3(pgrid), dim3(NT), 0, s, d_pairs, run,
                           p);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_geo_finish<TW, TH, CONN, NT, BOUND>), dim3(1), dim3(NT), 0, s, d_pairs, run, passes);
    return hipGetLastError();
}

template <int TW, int TH, int CONN, int NT>
hipError_t launch_t(const PairDev* d_pairs, const RunDev& run, int passes, hipStream_t s) {
    return run.total_tiles > kListTiles ? launch_l<TW, TH, CONN, NT, true>(d_pairs, run, passes, s)
                                        : launch_l<TW, TH, CONN, NT, false>(d_pairs, run, passes, s);
}

// Bounded transforms (32 x 16 tiles, default threads).
template <int CONN>
hipError_t launch_bounded(const PairDev* d_pairs, const RunDev& run, int passes, hipStream_t s) {
    return run.total_tiles > kListTiles ? launch_l<32, 16, CONN, 256, true, true>(d_pairs, run, passes, s)
                                        : launch_l<32, 16, CONN, 256, false, true>(d_pairs, run, passes, s);
}

// Threads per tile: runs of 2 pixels (32 x 16), 8 (32 x 32, 32 x 64)
constexpr int kThreads16 = 256, kThreads32 = 128, kThreads64 = 256;
}  // namespace

hipError_t launch_geodesic(const PairDev* d_pairs, const RunDev& run, int tile_w, int tile_h, int threads,
                           int passes, hipStream_t s) {
    const bool c8 = run.conn != 4;
    if (run.bounded) {
        if (tile_w != 32 || tile_h != 16) return hipErrorInvalidValue;
        return c8 ? launch_bounded<8>(d_pairs, run, passes, s) : launch_bounded<4>(d_pairs, run, passes, s);
    }
    if (tile_h == 16 && threads == 128)      // runs of 4 pixels in the later passes
        return c8 ? launch_t<32, 16, 8, 128>(d_pairs, run, passes, s)
                  : launch_t<32, 16, 4, 128>(d_pairs, run, passes, s);
    if (tile_h == 16)
        return c8 ? launch_t<32, 16, 8, kThreads16>(d_pairs, run, passes, s)
                  : launch_t<32, 16, 4, kThreads16>(d_pairs, run, passes, s);
    if (tile_h == 64)
        return c8 ? launch_t<32, 64, 8, kThreads64>(d_pairs, run, passes, s)
                  : launch_t<32, 64, 4, kThreads64>(d_pairs, run, passes, s);
    return c8 ? launch_t<32, 32, 8, kThreads32>(d_pairs, run, passes, s)
              : launch_t<32, 32, 4, kThreads32>(d_pairs, run, passes, s);
}

}  // namespace epic
