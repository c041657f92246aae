// k_graph.hip -- the match graph of Sec. 3.4 ("Approximated geodesic
// distance"): matches whose Voronoi cells touch are joined by an edge whose
// weight is the geodesic distance between the two matches restricted to
// their two cells.
//
// Because every cell is star-shaped around its match for the geodesic
// (each pixel's shortest path to its match stays in the cell), that
// restricted distance equals the minimum over adjacent pixel pairs (p in
// cell m, q in cell n) of D(p) + step(p, q) + D(q): every restricted path
// crosses from cell m to cell n a last time, and the two in-cell shortest
// paths joined by that step attain the bound.  So the graph is built by one
// scan over adjacent pixel pairs with a keyed minimum:
//   k_graph_emit     each pixel looks at its "forward" neighbours (right,
//                    down, and the two lower diagonals for 8-connectivity),
//                    so every unordered pair is seen once; pairs with
//                    different labels insert (min label, max label) into an
//                    open-addressing hash with an atomic min on the weight
//                    (positive floats order like their bits).  The first
//                    insertion of an edge raises both endpoints' degree.
//   k_csr_scan       one workgroup per pair: clamps K to the usable matches
//                    (counted by the seeding) and turns degrees into CSR row
//                    offsets.
//                    Every insertion also lowers both endpoints' lightest
//                    incident edge (the minimum over a node's candidates is
//                    the minimum over its edges).
//   k_csr_scatter    writes both directions of every edge into CSR.  Each
//                    record also carries the neighbour's CSR range and
//                    lightest incident edge, so the K-NN search learns all it
//                    needs about a newly reached node from the edge itself.
#include <type_traits>

#include "epic_dev.h"
#include "wave.h"

namespace epic {

namespace {
__device__ __forceinline__ u32 hash_slot(u64 key, int shift) {
    // 64-bit multiplicative mix (Fibonacci hashing of a murmur-style mix)
    key ^= key >> 33;
    key *= 0xff51afd7ed558ccdull;
    key ^= key >> 33;
    return (u32)((key * 0x9e3779b97f4a7c15ull) >> shift);
}
}  // namespace

namespace {
// Inserts (key, weight) into the pair's global hash with an atomic min on
// the weight; the first insertion of a key raises both endpoints' degree.
// Each probe is one compare-and-swap (it claims an empty slot or returns
// the key already there), so a slot costs one round trip, not a load and a
// swap.
template <bool F64>
__device__ __forceinline__ void global_insert(const PairDev& P, u64 hk, u64 wb) {
    const u32 mask = (u32)P.hash_cap - 1u;
    u32 h = hash_slot(hk, P.hash_shift);
    for (int probe = 0; probe < P.hash_cap; ++probe) {
        u64 cur = atomicCAS(&P.hkey[h], HASH_EMPTY, hk);
        if (cur == HASH_EMPTY) {
            atomicAdd(&P.deg[(u32)(hk >> 32)], 1u);
            atomicAdd(&P.deg[(u32)hk], 1u);
            cur = hk;
        }
        if (cur == hk) {
            const u32 m = (u32)(hk >> 32), n = (u32)hk;
            if (F64) {
                atomicMin(&P.hval64[h], wb);
                atomicMin(&P.minin64[m], wb);
                atomicMin(&P.minin64[n], wb);
            } else {
                atomicMin(&P.hval[h], (u32)wb);
                atomicMin(&P.minin[m], (u32)wb);
                atomicMin(&P.minin[n], (u32)wb);
            }
            return;
        }
        h = (h + 1u) & mask;
    }
    atomicOr(&P.counters[C_OVERFLOW], 1);
}
}  // namespace

// Each block handles one EMIT_TW x EMIT_TH tile of pixels.  Candidates are
// first reduced in a block-local LDS hash (adjacent pixels mostly share their
// pair of cells), then each distinct edge goes to the global hash once per
// block; a compact tile meets far fewer cell boundaries than a pixel strip of
// the same size, so few edges reach the global hash per block.  The occupied
// local slots are listed first, so the block's inserts run on distinct
// threads at once instead of in sequence on the threads that own several.
// PPT pixels per thread (rows y and y + EMIT_TH / PPT of the tile) with a
// local table PPT times smaller: more blocks fit a CU at once, which pays
// when the call has many tiles to keep the chip busy.
template <int CONN, bool F64, int PPT>
__global__ __launch_bounds__(EMIT_NT / PPT) void k_graph_emit(const PairDev* __restrict__ pairs, RunDev run) {
    constexpr int NT = EMIT_NT / PPT;                 // threads of the block
    constexpr int LCAP = EMIT_LCAP / PPT;             // block-local edge slots (overflow goes global)
    constexpr int LBITS = __builtin_ctz(LCAP);
    static_assert((1 << LBITS) == LCAP && LCAP <= 65536, "local hash: a power of two, 16-bit slot list");
    using V = typename std::conditional<F64, u64, u32>::type;
    __shared__ u64 lkey[LCAP];
    __shared__ V lval[LCAP];
    __shared__ unsigned short s_list[LCAP];
    __shared__ int s_cnt;
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].emit_block_base; });
    const PairDev& P = pairs[p];
    for (int i = threadIdx.x; i < LCAP; i += NT) {
        lkey[i] = HASH_EMPTY;
        lval[i] = F64 ? (V)DOUBLE_INF_BITS : (V)FLOAT_INF_BITS;
    }
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int W = P.W, H = P.H;
    const int tb = (int)blockIdx.x - P.emit_block_base, etx = (W + EMIT_TW - 1) / EMIT_TW;
#pragma unroll
    for (int pp = 0; pp < PPT; ++pp) {
        const int t = (int)threadIdx.x + pp * NT;         // pixel of the tile
        const int x = (tb % etx) * EMIT_TW + t % EMIT_TW;
        const int y = (tb / etx) * EMIT_TH + t / EMIT_TW;
        const long long i = (long long)y * W + x;
        if (x < W && y < H) {
            // forward half-neighbourhood: (1,0), (0,1), (1,1), (-1,1); all loads
            // are issued before any is used (outside neighbours read the pixel
            // itself and are skipped)
            constexpr int HX[4] = {1, 0, 1, -1};
            constexpr int HY[4] = {0, 1, 1, 1};
            constexpr int NK = CONN == 8 ? 4 : 2;
            const u64 kp = gmem(P.keys)[i];
            const float cp = gmem(P.cost)[i];
            const u32 lp = F64 ? gmem(P.labels)[i] : key_label(kp);
            u64 kqa[NK];
            float cqa[NK];
            u32 lqa[NK];
            bool in[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int qx = x + HX[k], qy = y + HY[k];
                in[k] = qx >= 0 && qx < W && qy < H;
                const long long qi = in[k] ? (long long)qy * W + qx : i;
                kqa[k] = gmem(P.keys)[qi];
                cqa[k] = gmem(P.cost)[qi];
                if (F64) lqa[k] = gmem(P.labels)[qi];
            }
            if (lp != NO_LABEL) {
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    if (!in[k]) continue;
                    const u64 kq = kqa[k];
                    const u32 lq = F64 ? lqa[k] : key_label(kq);
                    if (lq == lp || lq == NO_LABEL) continue;
                    V wb;
                    // (D(p) + step) + D(q), each operation rounded on its own (the
                    // helpers are never fused into multiply-adds)
                    if (F64) {
                        const double step = step_f64(cp, cqa[k], k < 2 ? 0 : 4);
                        wb = (V)bitsd(relax_f64(relax_f64(dbits(kp), step), dbits(kq)));
                    } else {
                        const float len = (k < 2) ? 1.0f : 1.41421356237309515f;
                        const float w = step_f32(len, cp, cqa[k]);
                        wb = (V)__float_as_uint(relax_f32(relax_f32(key_dist(kp), w), key_dist(kq)));
                    }
                    const u32 m = min(lp, lq), n = max(lp, lq);
                    const u64 hk = ((u64)m << 32) | n;
                    u32 h = (u32)(((hk ^ (hk >> 29)) * 0x9e3779b97f4a7c15ull) >> (64 - LBITS));
                    bool done = false;
                    for (int probe = 0; probe < LCAP; ++probe) {
                        const u64 prev = atomicCAS(&lkey[h], HASH_EMPTY, hk);
                        if (prev == HASH_EMPTY || prev == hk) {
                            atomicMin(&lval[h], wb);
                            done = true;
                            break;
                        }
                        h = (h + 1u) & (LCAP - 1);
                    }
                    if (!done) global_insert<F64>(P, hk, wb);
                }
            }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < LCAP; j += NT)
        if (lkey[j] != HASH_EMPTY) s_list[atomicAdd(&s_cnt, 1)] = (unsigned short)j;
    __syncthreads();
    const int cnt = s_cnt;
    for (int k = threadIdx.x; k < cnt; k += NT) {
        const int j = s_list[k];
        global_insert<F64>(P, lkey[j], lval[j]);
    }
}

// One workgroup of 1024 threads per pair.  Each thread sums a contiguous
// chunk of degrees (a multiple of 4, read as uint4), the chunk sums are
// scanned within each wavefront (DPP) and across the 16 wavefronts, and each
// thread writes its chunk's row offsets.
__global__ __launch_bounds__(1024) void k_csr_scan(const PairDev* __restrict__ pairs, RunDev run) {
    const PairDev& P = pairs[blockIdx.x];
    __shared__ u32 s_wave[16];
    __shared__ int s_big[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int N = P.N;
    const int chunk = ((N + 1023) / 1024 + 3) & ~3;
    const int b = min(N, tid * chunk), e = min(N, b + chunk);
    u32 sum = 0, dor = 0;    // dor: OR of the degrees (FP32 records hold 16 bits)
    if (e - b == chunk) {
        for (int m = b; m < e; m += 4) {
            const uint4 d = *reinterpret_cast<const uint4*>(P.deg + m);
            sum += d.x + d.y + d.z + d.w;
            dor |= d.x | d.y | d.z | d.w;
        }
    } else {
        for (int m = b; m < e; ++m) {
            sum += P.deg[m];
            dor |= P.deg[m];
        }
    }
    const u32 incl = (u32)wave::incl_scan((int)sum);
    const bool big = wave::ballot(dor > 0xffffu) != 0ull;
    if (lane == 63) {
        s_wave[wid] = incl;
        s_big[wid] = big ? 1 : 0;
    }
    __syncthreads();
    u32 base = 0;
    for (int w = 0; w < wid; ++w) base += s_wave[w];
    u32 run_sum = base + incl - sum;
    if (e - b == chunk) {
        for (int m = b; m < e; m += 4) {
            const uint4 d = *reinterpret_cast<const uint4*>(P.deg + m);
            uint4 o;
            o.x = run_sum;
            o.y = o.x + d.x;
            o.z = o.y + d.y;
            o.w = o.z + d.z;
            run_sum = o.w + d.w;
            *reinterpret_cast<uint4*>(P.row_ptr + m) = o;
        }
    } else {
        for (int m = b; m < e; ++m) {
            P.row_ptr[m] = run_sum;
            run_sum += P.deg[m];
        }
    }
    u32 two_e_total = 0;
    for (int w = 0; w < 16; ++w) two_e_total += s_wave[w];
    if (tid == 0) P.row_ptr[N] = two_e_total;
    if (tid == 0) {
        const int u = P.counters[C_USED];     // distinct seed pixels (counted by the seeding)
        P.counters[C_DUPLICATE] = N - P.counters[C_OUTSIDE] - u;
        P.counters[C_KEFF] = min(P.K, u);
        int status = 0;
        if (u == 0) status = -3;                                       // EPIC_ERR_NO_MATCHES
        const u32 two_e = two_e_total;        // every edge counted at both ends
        P.counters[C_EDGES] = (int)(two_e / 2);
        if ((long long)two_e > (long long)P.hash_cap) P.counters[C_OVERFLOW] |= 1;
        int any_big = 0;
        for (int w = 0; w < 16; ++w) any_big |= s_big[w];
        if (any_big && P.minin64 == nullptr) P.counters[C_OVERFLOW] |= 1;   // a degree above 65535
        if (P.counters[C_OVERFLOW]) status = -6;                       // EPIC_ERR_CAPACITY
        if ((*run.error & 1) || P.counters[C_GEOERR]) status = -7;     // EPIC_ERR_CONVERGENCE
        if (P.counters[C_BADCOST]) {                                   // EPIC_ERR_COST: not seeded
            status = -8;
            P.counters[C_DUPLICATE] = 0;
        }
        P.counters[C_STATUS] = status;
    }
}

__global__ __launch_bounds__(SLOT_BLOCK) void k_csr_scatter(const PairDev* __restrict__ pairs, RunDev run) {
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].slot_block_base; });
    const PairDev& P = pairs[p];
    const int h = ((int)blockIdx.x - P.slot_block_base) * SLOT_BLOCK + threadIdx.x;
    if (h >= P.hash_cap) return;
    const u64 key = gmem(P.hkey)[h];
    if (key == HASH_EMPTY) return;
    const u32 m = (u32)(key >> 32), n = (u32)key;
    const bool f64 = run.precision == 1;
    const u32 wb = f64 ? __float_as_uint((float)dbits(gmem(P.hval64)[h])) : gmem(P.hval)[h];
    const float w = __uint_as_float(wb);
    const u32 rm = gmem(P.row_ptr)[m], rm1 = gmem(P.row_ptr)[m + 1];
    const u32 rn = gmem(P.row_ptr)[n], rn1 = gmem(P.row_ptr)[n + 1];
    const u32 pm = rm + atomicAdd(&P.fill[m], 1u);
    const u32 pn = rn + atomicAdd(&P.fill[n], 1u);
    const bool okm = pm < (u32)P.hash_cap, okn = pn < (u32)P.hash_cap;
    // FP32 path: the neighbour's degree (below 2^16, checked by the scan) and
    // its lightest edge truncated to 16 bits (a lower bound) share a word
    const u32 wn = f64 ? rn1 - rn : (rn1 - rn) | (gmem(P.minin)[n] & 0xffff0000u);
    const u32 wm = f64 ? rm1 - rm : (rm1 - rm) | (gmem(P.minin)[m] & 0xffff0000u);
    if (okm) gstore(P.adj + pm, make_uint4(n, wb, rn, wn));
    if (okn) gstore(P.adj + pn, make_uint4(m, wb, rm, wm));
    if (f64) {
        const u64 wd = gmem(P.hval64)[h];
        if (okm) {
            gmem(P.adjw64)[pm] = dbits(wd);
            gmem(P.nbmin64)[pm] = gmem(P.minin64)[n];
        }
        if (okn) {
            gmem(P.adjw64)[pn] = dbits(wd);
            gmem(P.nbmin64)[pn] = gmem(P.minin64)[m];
        }
    }
    if (P.dbg_em) {
        const int e = atomicAdd(P.dbg_n_edges, 1);
        if (e < P.dbg_max_edges) {
            P.dbg_em[e] = (int)m;
            P.dbg_en[e] = (int)n;
            P.dbg_ew[e] = w;
        }
    }
}

hipError_t launch_graph_emit(const PairDev* d_pairs, const RunDev& run, int total_blocks, long long total_px,
                             hipStream_t s) {
    const bool f64 = run.precision == 1;
    // two pixels per thread once the call has at least 2.1 Mpx (the tiles of
    // four full chips of one-pixel threads)
    const bool two = total_px >= 4LL * 256 * 32 * 64;
    const dim3 b1(EMIT_NT), b2(EMIT_NT / 2);
    if (run.conn == 4) {
        if (f64) {
            if (two) hipLaunchKernelGGL((k_graph_emit<4, true, 2>), dim3(total_blocks), b2, 0, s, d_pairs, run);
            else hipLaunchKernelGGL((k_graph_emit<4, true, 1>), dim3(total_blocks), b1, 0, s, d_pairs, run);
        } else {
            if (two) hipLaunchKernelGGL((k_graph_emit<4, false, 2>), dim3(total_blocks), b2, 0, s, d_pairs, run);
            else hipLaunchKernelGGL((k_graph_emit<4, false, 1>), dim3(total_blocks), b1, 0, s, d_pairs, run);
        }
    } else {
        if (f64) {
            if (two) hipLaunchKernelGGL((k_graph_emit<8, true, 2>), dim3(total_blocks), b2, 0, s, d_pairs, run);
            else hipLaunchKernelGGL((k_graph_emit<8, true, 1>), dim3(total_blocks), b1, 0, s, d_pairs, run);
        } else {
            if (two) hipLaunchKernelGGL((k_graph_emit<8, false, 2>), dim3(total_blocks), b2, 0, s, d_pairs, run);
            else hipLaunchKernelGGL((k_graph_emit<8, false, 1>), dim3(total_blocks), b1, 0, s, d_pairs, run);
        }
    }
    return hipGetLastError();
}

hipError_t launch_csr_scan(const PairDev* d_pairs, const RunDev& run, hipStream_t s) {
    hipLaunchKernelGGL(k_csr_scan, dim3(run.npairs), dim3(1024), 0, s, d_pairs, run);
    return hipGetLastError();
}

hipError_t launch_csr_scatter(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_csr_scatter, dim3(total_blocks), dim3(SLOT_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

}  // namespace epic
