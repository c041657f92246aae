// epic_dev.h -- shared device-side definitions of the interpolation library:
// the per-pair descriptor that every kernel reads, key packing, and the
// host-side launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

typedef unsigned long long u64;
typedef unsigned int u32;

// A pixel's transform state is one 64-bit key: the float bits of the geodesic
// distance D in the high word and the match label in the low word.  D >= 0,
// so the float bits order like the values, and the unsigned order of keys is
// the lexicographic order on (D, label): a lexicographic min is one integer
// min, and ties in D go to the lowest label.
constexpr u64 KEY_INF = 0x7f800000ffffffffull;   // (+inf, no label)
constexpr u32 NO_LABEL = 0xffffffffu;
constexpr u64 HASH_EMPTY = ~0ull;
constexpr u32 FLOAT_INF_BITS = 0x7f800000u;
constexpr u64 DOUBLE_INF_BITS = 0x7ff0000000000000ull;

__device__ __forceinline__ double dbits(u64 k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ u64 bitsd(double d) { return (u64)__double_as_longlong(d); }

__device__ __forceinline__ float key_dist(u64 k) { return __uint_as_float((u32)(k >> 32)); }
__device__ __forceinline__ u32 key_label(u64 k) { return (u32)k; }
__device__ __forceinline__ u64 make_key(float d, u32 label) {
    return ((u64)__float_as_uint(d) << 32) | (u64)label;
}

// Per-pair counters (int32 each).
enum Counter {
    C_STATUS = 0,      // epic_status found on the device
    C_USED = 1,
    C_OUTSIDE = 2,
    C_DUPLICATE = 3,
    C_EDGES = 4,
    C_DEGENERATE = 5,
    C_FP64 = 6,
    C_KEFF = 7,        // K clamped to the usable matches
    C_OVERFLOW = 8,    // bit 0 graph hash, bit 1 Dijkstra visited table
    C_TILE_VISITS = 9,
    C_BADCOST = 10,    // cost values not finite and > 0 (checked on request)
    C_GEOERR = 11,     // a transform visit of this pair hit its round bound
    // kept across the two passes of a call with the consistency check (the
    // second pass clears only the counters before C_PRUNED)
    C_PRUNED = 12,     // placed matches removed by the consistency check
    C_OUTSIDE0 = 13,   // the first pass's outside / duplicate counts and status
    C_DUP0 = 14,
    C_STATUS0 = 15,
    C_INVARIANT = 16,  // debug_validate: violated invariants of the transform and graph
    // bounded transforms: the tiles a pair's distances reached, as a box
    // (0 = none): (1 << 24) - least tile x / y, 1 + greatest tile x / y
    C_BX0 = 17,
    C_BY0 = 18,
    C_BX1 = 19,
    C_BY1 = 20,
    C_NCOUNTERS = 21
};

// Everything a kernel needs about one image pair.  Kernels of a batch launch
// receive an array of these and find their pair from their work-item index.
struct PairDev {
    // inputs / output (caller-owned)
    const float* cost;      // H*W
    const float* matches;   // N*4
    float* flow;            // H*W*2
    int H, W, N, K;
    float a;
    int mode;
    // work decomposition (global index bases across the batch)
    int tiles_x, tiles_y;
    int tile_base;          // first global tile id of this pair
    int pix_block_base;     // first block of pixel-parallel grids (a multiple of
                            //   ASSIGN_PPT: the assignment's grid, ASSIGN_PPT times
                            //   coarser, starts the pair at pix_block_base / ASSIGN_PPT)
    int emit_block_base;    // first block of the graph-emit grid (EMIT_TW x EMIT_TH tiles)
    int src_block_base;     // first block of the per-match grid (one match per block)
    int seed_block_base;    // first block of the seeding grid (PIX_BLOCK matches per block)
    int slot_block_base;    // first block of the hash-slot grid
    int init_block_base;    // first block of the clearing grid
    int init_blocks;        // blocks of the clearing grid for this pair
    int hash_cap;           // power of two
    int hash_shift;         // 64 - log2(hash_cap)
    // workspace (context-owned)
    u64* keys;              // H*W transform state
    int* seed_pix;          // N: seed pixel of a match, -1 when outside
    u64* hkey;              // hash_cap: (m << 32 | n), m < n
    u32* hval;              // hash_cap: float bits of the edge weight
    u32* deg;               // N
    u32* fill;              // N (CSR fill counts; in the first pass of the
                            //   consistency check the K-NN then stores each match's
                            //   keep flag there, the counts being used up)
    u32* row_ptr;           // N + 1
    u32* minin;             // N: float bits of the lightest incident edge
    uint4* adj;             // hash_cap: CSR edges (neighbour id, weight bits,
                            //   neighbour's CSR start, neighbour's degree in the low
                            //   16 bits and the high 16 bits of its lightest edge's
                            //   float bits in the high 16; FP64 path: the degree alone)
    float* params;          // N*6
    int* counters;          // C_NCOUNTERS
    // FP64-everywhere path only (NULL otherwise)
    u32* labels;            // H*W nearest-match label (keys then hold double D)
    u64* hval64;            // hash_cap: double bits of the edge weight
    u64* minin64;           // N: double bits of the lightest incident edge
    double* adjw64;         // hash_cap: CSR edge weights
    u64* nbmin64;           // hash_cap: double bits of the neighbour's lightest edge
    double* params64;       // N*6
    // consistency check of the matches (Sec. 5.1): the kept matches,
    // compacted in index order, and their original indices
    // exact interpolation: per-pixel bound on the distances worth keeping in
    // a single-source transform (null: none)
    const float* ubound;    // H*W
    // bounded runs: the only pixels whose keys the clearing must reset (the
    // box the pair that last used this workspace reached; null = all)
    const int4* clear_box;
    float* matches_kept;    // N*4
    int* kept_idx;          // N
    // optional stage dumps (NULL = off)
    int* dbg_knn_idx;       // N*K
    float* dbg_knn_d;       // N*K
    int* dbg_em;            // max_edges
    int* dbg_en;
    float* dbg_ew;
    int dbg_max_edges;
    int* dbg_n_edges;       // device int
    int* dbg_kept;          // N: original indices of the kept matches
    int* dbg_n_kept;        // device int
};

// Global-memory view of a pointer.  Pointers read out of a PairDev (which
// lives in device memory) are generic to the compiler, which then emits flat
// memory instructions: those also count on the LDS counter, so every wait for
// a load waits for outstanding LDS traffic too, and they need 64-bit VGPR
// addresses.  Through an address-space-1 pointer the loads and stores are
// global instructions.
#define EPIC_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ EPIC_GLOBAL T* gmem(T* p) { return (EPIC_GLOBAL T*)p; }
// The HIP vector classes cannot be copied from or to address-space-1
// objects; these go through the compiler's own vector types.
typedef unsigned int gu32x4 __attribute__((ext_vector_type(4)));
typedef float gf32x4 __attribute__((ext_vector_type(4)));
typedef float gf32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 gload(const uint4* p) {
    const gu32x4 v = *(const EPIC_GLOBAL gu32x4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 gload(const float4* p) {
    const gf32x4 v = *(const EPIC_GLOBAL gf32x4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gload(const float2* p) {
    const gf32x2 v = *(const EPIC_GLOBAL gf32x2*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gstore(uint4* p, uint4 v) { *(EPIC_GLOBAL gu32x4*)p = gu32x4{v.x, v.y, v.z, v.w}; }
__device__ __forceinline__ void gstore(float2* p, float2 v) { *(EPIC_GLOBAL gf32x2*)p = gf32x2{v.x, v.y}; }
__device__ __forceinline__ void gstore(float4* p, float4 v) {
    *(EPIC_GLOBAL gf32x4*)p = gf32x4{v.x, v.y, v.z, v.w};
}

// Relaxed atomic accesses for transform state that other threads read or
// write at the same moment.  The transform's correctness argument only
// needs each 64-bit (D, label) key to be read and written whole (a reader
// sees the old or the new key, never a mix: a torn key could pair a new
// distance with an old label and order below the optimum).  Relaxed atomics
// state exactly that and nothing more (no ordering, no fences):
//   lds_*     keys and flags in LDS shared by the waves of one workgroup
//             (plain ds_read_b64 / ds_write_b64);
//   dev_*     keys in global memory that workgroups of the same launch read
//             as halo while their owner writes them (agent scope).
template <typename T>
__device__ __forceinline__ T lds_ld(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void lds_st(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ T dev_ld(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void dev_st(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One step of the discretised geodesic of Eq. (3) in FP32, and a relaxation
// across it, each operation rounded on its own, so that every place that
// prices a step gets the same bits.  HIP's __fmul_rn / __fadd_rn are plain
// operators that the compiler may fuse into a multiply-add once inlined
// (relax_f32(d, step_f32(...)) in one expression would become an FMA in one
// kernel and a multiply and an add in another); the pragma keeps these
// operations unfused wherever they are inlined.
__device__ __forceinline__ float step_f32(float len, float cp, float cq) {
#pragma clang fp contract(off)
    return len * (0.5f * (cp + cq));
}
__device__ __forceinline__ float relax_f32(float d, float w) {
#pragma clang fp contract(off)
    return d + w;
}
// The same step in FP64 (the FP64-everywhere transform): neighbour k < 4 is
// axial, k >= 4 diagonal; relax_f64 adds it.
__device__ __forceinline__ double step_f64(float cp, float cq, int k) {
#pragma clang fp contract(off)
    const double half = 0.5 * ((double)cp + (double)cq);
    return k < 4 ? half : 1.4142135623730951 * half;
}
__device__ __forceinline__ double relax_f64(double d, double w) {
#pragma clang fp contract(off)
    return d + w;
}

// Nearest-match label of pixel i (packed in the key, or in the label array
// of the FP64 path).
__device__ __forceinline__ u32 label_at(const PairDev& P, long long i) {
    return P.labels ? P.labels[i] : key_label(P.keys[i]);
}

// Globals of one launch sequence (shared by all pairs of a batch).
struct RunDev {
    u32* dirty[2];          // per tile, by pass parity: tile needs a visit
    u32* wl[3];             // the dirty tiles of pass p, listed in wl[p % 3] (FP32
                            //   transform): each tile once, appended when its flag is set
    int* wl_cnt;            // 3 list lengths
    int* any;               // per pass: some tile border changed (kMaxPasses)
    int* any2;              // the same for the label phase of the FP64 path
    int* pass_visits;       // per pass: tile visits of the FP32 transform (counted
                            //   only while profiling; null otherwise)
    int* error;             // global error word: bit 0 = the transform finisher hit
                            //   its pass bound (per-pair errors live in the counters)
    int* passes_used;       // host-visible, 2 ints: passes the last transform needed
                            //   (FP64 path: distance phase, label phase); may be null
    int* ovf_list;          // K-NN sources to redo with a larger table
    int* ovf_count;
    int total_tiles;
    int npairs;
    int conn;               // 8 or 4
    int tile_w, tile_h;     // geodesic-transform tile
    int la_wpow;            // 1 or 2
    int precision;          // 0 or 1
    float fp64_route;
    double deg_tau;
    int bounded;            // 1: the transform keeps only distances within P.ubound
    int force_nw;           // 1: fit NW whatever the pair's mode (the first pass of
                            //   the consistency check)
    int keep_prune_counters;   // 1: the clear keeps counters C_PRUNED.. (second pass)
    float prune_px;         // > 0 in the first pass of the consistency check: the
                            //   K-NN + fit writes each match's keep flag into fill[]
};

constexpr int kMaxPasses = 256;  // passes launched per call, at most (pass flags
                                 //   live in the workspace's first 4 KiB)

// Descriptor tables of up to kInlinePairs pairs travel in the first kernel's
// arguments (which the launch copies anyway); that kernel writes them to the
// device table the later kernels read.  Larger tables are uploaded with a copy.
constexpr int kInlinePairs = 8;
struct DescInline {
    int n;                          // 0: the device table is already uploaded
    PairDev p[kInlinePairs];
};

// Binary search: the pair whose base <= idx (bases ascending).
template <typename F>
__device__ __forceinline__ int find_pair(int npairs, int idx, F base_of) {
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base_of(mid) <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// host-side launchers (one per stage; defined next to their kernels)
// ---------------------------------------------------------------------------
constexpr int PIX_BLOCK = 256;      // pixels per block of pixel-parallel kernels
constexpr int ASSIGN_PPT = 4;      // pixels per thread of the assignment on calls with many pixels
constexpr int EMIT_TW = 32, EMIT_TH = 16;  // pixel tile of one graph-emit block
constexpr int EMIT_NT = EMIT_TW * EMIT_TH; // one thread per pixel
constexpr int EMIT_LCAP = 4 * EMIT_NT;     // block-local edge slots
constexpr int SLOT_BLOCK = 256;     // hash slots per block

hipError_t launch_clear(const PairDev* d_pairs, const RunDev& run, int total_blocks, const PairDev* inline_host,
                        int n_inline, hipStream_t s);
hipError_t launch_seed(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s);
hipError_t launch_check_cost(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s);
hipError_t launch_geodesic(const PairDev* d_pairs, const RunDev& run, int tile_w, int tile_h, int threads,
                           int passes, hipStream_t s);
hipError_t launch_geodesic64(const PairDev* d_pairs, const RunDev& run, int passes0, int passes1, hipStream_t s);
hipError_t launch_graph_emit(const PairDev* d_pairs, const RunDev& run, int total_blocks, long long total_px,
                             hipStream_t s);
hipError_t launch_csr_scan(const PairDev* d_pairs, const RunDev& run, hipStream_t s);
hipError_t launch_csr_scatter(const PairDev* d_pairs, const RunDev& run, int total_blocks, hipStream_t s);
hipError_t launch_knn_fit(const PairDev* d_pairs, const RunDev& run, int total_blocks, int kmax, int nmax,
                          hipStream_t s);
hipError_t launch_assign(const PairDev* d_pairs, const RunDev& run, int pix_blocks, long long total_px,
                         hipStream_t s);
hipError_t launch_prune(PairDev* d_pairs, const RunDev& run, hipStream_t s);

// Cost map from the image gradient: up to kImagesPerLaunch images per launch,
// described in the kernel arguments.
struct ImageDesc {
    const float* image;     // H*W*channels, interleaved
    float* cost;            // H*W
    int H, W;
    int block_base;         // first block of this image's strips
    int pad;
};
constexpr int kImagesPerLaunch = 64;
struct ImageCostArgs {
    ImageDesc img[kImagesPerLaunch];
    int n;
    float eps;
};
int image_cost_blocks(int H, int W);

// Exact per-pixel geodesic interpolation (every pixel's own K nearest
// matches under the geodesic distance itself).
struct ExactArgs {
    const float* matches;   // N*4, the call's matches
    int N, K, H, W;
    long long HW;
    u64* lists;             // K*HW: entry k of pixel p at k*HW + p, packed
                            //   (distance bits << 32 | match), ascending; ~0 = none
    unsigned char* owner;   // N: 1 when the match holds its pixel
    float* ubound;          // H*W: bound on the distance of the pixel's K-th nearest match
    int* knn_idx;           // N*K: the approximated K-NN lists the bound comes from
    float* knn_d;           // N*K
    int4* boxes;            // per source of a chunk: the pixel box its transform reached
                            //   (empty for sources that hold no pixel)
    int4* clear_boxes;      // the same for every source (what the next chunk must clear)
    float* flow;            // H*W*2
    float a;
    int mode, wpow;
    float fp64_route;
    double deg_tau;
};
hipError_t launch_exact_owner(const PairDev* full, const ExactArgs& A, hipStream_t s);
hipError_t launch_exact_select(const PairDev* chunk, int nsrc, int src0, int first, int last, const ExactArgs& A,
                               hipStream_t s);
hipError_t launch_exact_fit(const ExactArgs& A, hipStream_t s);
hipError_t launch_exact_bound(const PairDev* full, const ExactArgs& A, hipStream_t s);
constexpr int kExactChunk = 1024;   // sources per chunk of the exact interpolation, at most
hipError_t launch_image_cost(const ImageCostArgs& args, int channels, int total_blocks, hipStream_t s);
hipError_t launch_check_transform(const PairDev* d_pairs, const RunDev& run, int pix_blocks, int plant,
                                  hipStream_t s);
hipError_t launch_check_graph(const PairDev* d_pairs, const RunDev& run, int slot_blocks, hipStream_t s);

// One-level variational refinement of a flow field (Sec. 4).
struct VarArgs {
    const float* I1;        // H*W*C, interleaved
    const float* I2;        // H*W*C
    const float* u0;        // H*W*2, the field to refine
    float* flow;            // H*W*2 output (may equal u0)
    float* I2w;             // H*W*C scratch: I2 warped by u0
    float* coef;            // 13 planes of H*W: JC (6), JG (6), alpha
    float* sys;             // 9 planes of H*W: a fixed-point step's per-pixel update
    float* du[2];           // H*W each, a ping-pong pair
    float* dv[2];
    int H, W, C;
    long long HW;
    float lam, delta, gamma, kappa, eps, zeta, omega;
    int fixed_point, sor;
};
constexpr int kVarPlanes = 13 + 9 + 4;   // float planes of H*W besides I2w
hipError_t launch_variational(const VarArgs& A, hipStream_t s);
hipError_t launch_unpack(const PairDev* d_pairs, const RunDev& run, int total_blocks, float* D, int* L,
                         hipStream_t s);

}  // namespace epic
