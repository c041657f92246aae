// k_prep.hip -- per-call workspace clearing, the optional check of the cost
// map, and match seeding.
//
// Seeding places every match on the pixel that contains it (matches are
// pixels, Sec. 3.1 of the paper): pixel (floor(x+0.5), floor(y+0.5)), decided
// in double precision.  Matches outside the image are dropped; when several
// matches fall on one pixel, the 64-bit atomic min on the packed key
// (D = 0, label) keeps the lowest match index, and the match that claims an
// empty pixel counts it (usable matches = distinct seed pixels).  The tile holding a seed is
// marked dirty for the geodesic transform.
#include "epic_dev.h"

namespace epic {

// Clears the per-pair workspace with grid-stride loops; each pair owns
// init_blocks consecutive blocks of the grid.  With an inline descriptor
// table, the descriptors come from the arguments and block 0 also writes
// them to the device table.
__global__ __launch_bounds__(256) void k_clear(PairDev* __restrict__ pairs, RunDev run, DescInline inl) {
    const PairDev* table = inl.n > 0 ? inl.p : pairs;
    if (inl.n > 0 && blockIdx.x == 0) {
        const u32* src = reinterpret_cast<const u32*>(inl.p);
        EPIC_GLOBAL u32* dst = reinterpret_cast<EPIC_GLOBAL u32*>(gmem(pairs));
        const int words = inl.n * (int)(sizeof(PairDev) / 4);
        for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
    }
    const int p = find_pair(run.npairs, (int)blockIdx.x,
                            [&](int i) { return table[i].init_block_base; });
    const PairDev& P = table[p];
    const int lb = (int)blockIdx.x - P.init_block_base;
    const long long stride = (long long)P.init_blocks * blockDim.x;
    const long long i0 = (long long)lb * blockDim.x + threadIdx.x;
    const long long HW = (long long)P.H * P.W;
    const bool f64 = run.precision == 1;
    if (P.clear_box) {
        // a bounded single-source run: only the box the previous user of
        // this workspace reached holds other values than infinity
        const int4 b = *P.clear_box;
        if (b.x <= b.z) {
            const int bw = b.z - b.x + 1;
            const long long nb = (long long)bw * (b.w - b.y + 1);
            for (long long i = i0; i < nb; i += stride)
                P.keys[(long long)(b.y + (int)(i / bw)) * P.W + b.x + (int)(i % bw)] = KEY_INF;
        }
    } else {
        for (long long i = i0; i < HW; i += stride) {
            P.keys[i] = f64 ? DOUBLE_INF_BITS : KEY_INF;
            if (f64) P.labels[i] = NO_LABEL;
        }
    }
    for (long long i = i0; i < P.hash_cap; i += stride) {
        P.hkey[i] = HASH_EMPTY;
        P.hval[i] = FLOAT_INF_BITS;
        if (f64) P.hval64[i] = DOUBLE_INF_BITS;
    }
    for (long long i = i0; i < P.N; i += stride) {
        P.deg[i] = 0u;
        P.fill[i] = 0u;
        P.minin[i] = FLOAT_INF_BITS;
        if (f64) P.minin64[i] = DOUBLE_INF_BITS;
    }
    const int ntiles = P.tiles_x * P.tiles_y;
    for (long long i = i0; i < ntiles; i += stride) {
        run.dirty[0][P.tile_base + i] = 0u;
        run.dirty[1][P.tile_base + i] = 0u;
    }
    if (i0 < (run.keep_prune_counters ? (long long)C_PRUNED : (long long)C_NCOUNTERS)) P.counters[i0] = 0;
    if (i0 == 0 && P.dbg_n_edges) *P.dbg_n_edges = 0;
    if (p == 0 && i0 < kMaxPasses) {
        run.any[i0] = 0;
        run.any2[i0] = 0;
        if (run.pass_visits) run.pass_visits[i0] = 0;
    }
    if (p == 0 && i0 == 0) {
        *run.error = 0;
        *run.ovf_count = 0;
    }
    if (p == 0 && i0 < 3) run.wl_cnt[i0] = 0;
}

__global__ __launch_bounds__(256) void k_seed(const PairDev* __restrict__ pairs, RunDev run) {
    const int p = find_pair(run.npairs, (int)blockIdx.x,
                            [&](int i) { return pairs[i].seed_block_base; });
    const PairDev& P = pairs[p];
    const int m = ((int)blockIdx.x - P.seed_block_base) * blockDim.x + threadIdx.x;
    const bool rejected = P.counters[C_BADCOST] != 0;   // the cost map failed its check
    int pix = -1;
    bool first = false;        // this match claimed an empty pixel
    if (m < P.N) {
        const double x = P.matches[4LL * m + 0];
        const double y = P.matches[4LL * m + 1];
        if (!rejected && isfinite(x) && isfinite(y)) {
            const double fx = floor(x + 0.5), fy = floor(y + 0.5);
            if (fx >= 0.0 && fy >= 0.0 && fx < (double)P.W && fy < (double)P.H) {
                const int ix = (int)fx, iy = (int)fy;
                pix = iy * P.W + ix;
                if (run.precision == 1) {
                    P.keys[pix] = 0ull;                      // D = 0.0 (double bits)
                    first = atomicMin(&P.labels[pix], (u32)m) == NO_LABEL;
                } else {
                    first = atomicMin(&P.keys[pix], make_key(0.0f, (u32)m)) == KEY_INF;
                }
                const int t = P.tile_base + (iy / run.tile_h) * P.tiles_x + ix / run.tile_w;
                run.dirty[0][t] = 1u;
            }
        }
        P.seed_pix[m] = pix;
    }
    // the usable matches are the lowest-indexed ones of the distinct seed
    // pixels, counted by their first claims; one counter update per
    // wavefront (updates of one address from every thread serialise)
    const u64 nf = __builtin_amdgcn_ballot_w64(first);
    const u64 no = __builtin_amdgcn_ballot_w64(m < P.N && pix < 0 && !rejected);
    if ((threadIdx.x & 63) == 0) {
        if (nf) atomicAdd(&P.counters[C_USED], (int)__popcll(nf));
        if (no) atomicAdd(&P.counters[C_OUTSIDE], (int)__popcll(no));
    }
}

// Optional check of the cost map: counts the values that are not finite and
// > 0 (one counter update per wavefront).  A nonzero count makes the seeding
// place no match of that pair.
__global__ __launch_bounds__(PIX_BLOCK) void k_check_cost(const PairDev* __restrict__ pairs, RunDev run) {
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].pix_block_base; });
    const PairDev& P = pairs[p];
    const long long i = (long long)((int)blockIdx.x - P.pix_block_base) * PIX_BLOCK + threadIdx.x;
    bool bad = false;
    if (i < (long long)P.W * P.H) {
        const float c = gmem(P.cost)[i];
        bad = !(c > 0.0f && c <= 3.402823466e38f);   // NaN, zero, negative or infinite
    }
    const u64 b = __builtin_amdgcn_ballot_w64(bad);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&P.counters[C_BADCOST], (int)__popcll(b));
}

hipError_t launch_check_cost(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_check_cost, dim3(total_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

hipError_t launch_clear(const PairDev* d_pairs, const RunDev& run, int total_blocks, const PairDev* inline_host,
                        int n_inline, hipStream_t s) {
    DescInline inl;
    inl.n = inline_host ? n_inline : 0;
    if (inl.n > kInlinePairs) return hipErrorInvalidValue;
    for (int i = 0; i < inl.n; ++i) inl.p[i] = inline_host[i];
    hipLaunchKernelGGL(k_clear, dim3(total_blocks), dim3(256), 0, s, const_cast<PairDev*>(d_pairs), run, inl);
    return hipGetLastError();
}

hipError_t launch_seed(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_seed, dim3(total_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

}  // namespace epic
