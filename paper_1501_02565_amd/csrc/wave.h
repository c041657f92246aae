// wave.h -- wavefront-wide reductions and scans for 64-lane waves on gfx950,
// built from DPP row operations (quad permutes, row mirrors, row shifts and
// the row broadcasts of GFX9) and a final readlane.  They stay in registers
// (no LDS traffic) and combine lanes in a fixed order, so results are
// deterministic.  All 64 lanes must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace epic {
namespace wave {

typedef unsigned long long u64_t;

// DPP controls (GFX9 encoding)
constexpr int QP_XOR1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int QP_XOR2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int ROW_HALF_MIRROR = 0x141;
constexpr int ROW_MIRROR = 0x140;
constexpr int ROW_SHR1 = 0x111, ROW_SHR2 = 0x112, ROW_SHR4 = 0x114, ROW_SHR8 = 0x118;
constexpr int ROW_SHL4 = 0x104, ROW_ROR8 = 0x128;
constexpr int ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;

template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ int dpp(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dppf(float old, float v) {
    return __int_as_float(dpp<CTRL, ROWMASK>(__float_as_int(old), __float_as_int(v)));
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dppd(double old, double v) {
    const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
    const int lo = dpp<CTRL, ROWMASK>((int)(o & 0xffffffff), (int)(x & 0xffffffff));
    const int hi = dpp<CTRL, ROWMASK>((int)(o >> 32), (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float readlane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double readlane63(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, returned to every lane.  Only lane 63 is read at
// the end, so the row broadcasts run on all rows (rows 0-2 may end up
// holding partial or doubled sums; row 3 gets rows 0 + 1, then 2, exactly
// once) and every step is one DPP add with out-of-row reads giving 0.
__device__ __forceinline__ float sum(float v) {
    v += dppf<QP_XOR1>(0.0f, v);
    v += dppf<QP_XOR2>(0.0f, v);
    v += dppf<ROW_HALF_MIRROR>(0.0f, v);
    v += dppf<ROW_MIRROR>(0.0f, v);          // every lane: its row's sum
    v += dppf<ROW_BCAST15>(0.0f, v);         // row 3 += row 2 (row 1 += row 0)
    v += dppf<ROW_BCAST31>(0.0f, v);         // row 3 += row 1
    return readlane63(v);
}
__device__ __forceinline__ double sum(double v) {
    v += dppd<QP_XOR1>(0.0, v);
    v += dppd<QP_XOR2>(0.0, v);
    v += dppd<ROW_HALF_MIRROR>(0.0, v);
    v += dppd<ROW_MIRROR>(0.0, v);
    v += dppd<ROW_BCAST15>(0.0, v);
    v += dppd<ROW_BCAST31>(0.0, v);
    return readlane63(v);
}
__device__ __forceinline__ int sum(int v) {
    v += dpp<QP_XOR1>(0, v);
    v += dpp<QP_XOR2>(0, v);
    v += dpp<ROW_HALF_MIRROR>(0, v);
    v += dpp<ROW_MIRROR>(0, v);
    v += dpp<ROW_BCAST15, 0xA>(0, v);
    v += dpp<ROW_BCAST31, 0xC>(0, v);
    return __builtin_amdgcn_readlane(v, 63);
}

// Minimum over the 64 lanes, returned to every lane.
__device__ __forceinline__ float min(float v) {
    const float inf = __int_as_float(0x7f800000);
    v = fminf(v, dppf<QP_XOR1>(inf, v));
    v = fminf(v, dppf<QP_XOR2>(inf, v));
    v = fminf(v, dppf<ROW_HALF_MIRROR>(inf, v));
    v = fminf(v, dppf<ROW_MIRROR>(inf, v));
    v = fminf(v, dppf<ROW_BCAST15, 0xA>(inf, v));
    v = fminf(v, dppf<ROW_BCAST31, 0xC>(inf, v));
    return readlane63(v);
}
__device__ __forceinline__ double min(double v) {
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    v = fmin(v, dppd<QP_XOR1>(inf, v));
    v = fmin(v, dppd<QP_XOR2>(inf, v));
    v = fmin(v, dppd<ROW_HALF_MIRROR>(inf, v));
    v = fmin(v, dppd<ROW_MIRROR>(inf, v));
    v = fmin(v, dppd<ROW_BCAST15, 0xA>(inf, v));
    v = fmin(v, dppd<ROW_BCAST31, 0xC>(inf, v));
    return readlane63(v);
}

// Inclusive prefix sum over lanes 0..63.
__device__ __forceinline__ int incl_scan(int v) {
    v += dpp<ROW_SHR1>(0, v);
    v += dpp<ROW_SHR2>(0, v);
    v += dpp<ROW_SHR4>(0, v);
    v += dpp<ROW_SHR8>(0, v);                 // scan within each row of 16
    v += dpp<ROW_BCAST15, 0xA>(0, v);
    v += dpp<ROW_BCAST31, 0xC>(0, v);
    return v;
}

// Inclusive prefix maximum over lanes 0..63 of unsigned values (0 is
// neutral, so every step is one DPP-fused maximum).
__device__ __forceinline__ unsigned incl_max(unsigned v) {
    v = max(v, (unsigned)dpp<ROW_SHR1>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_SHR2>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_SHR4>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_SHR8>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_BCAST15, 0xA>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_BCAST31, 0xC>(0, (int)v));
    return v;
}

// Maximum of unsigned values over the 64 lanes, returned to every lane.
__device__ __forceinline__ unsigned max_u32(unsigned v) {
    v = max(v, (unsigned)dpp<QP_XOR1>(0, (int)v));
    v = max(v, (unsigned)dpp<QP_XOR2>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_HALF_MIRROR>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_MIRROR>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_BCAST15, 0xA>(0, (int)v));
    v = max(v, (unsigned)dpp<ROW_BCAST31, 0xC>(0, (int)v));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Minimum of non-negative floats (or +inf) over the 64 lanes: their bits
// order like the values, and min = ~max(~bits) keeps the neutral value 0.
__device__ __forceinline__ float min_nonneg(float v) {
    return __uint_as_float(~max_u32(~__float_as_uint(v)));
}

__device__ __forceinline__ u64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// The value held by lane (this lane xor J), J a power of two below 64:
// quad permutes for 1 and 2, row shifts that write alternate groups of four
// lanes for 4, a half-row rotation for 8, a swizzle within 32 lanes for 16
// and a lane permute for 32.
template <int J>
__device__ __forceinline__ int xor_lane(int v) {
    static_assert(J == 1 || J == 2 || J == 4 || J == 8 || J == 16 || J == 32, "lane distance");
    if constexpr (J == 1) {
        return __builtin_amdgcn_mov_dpp(v, QP_XOR1, 0xF, 0xF, false);
    } else if constexpr (J == 2) {
        return __builtin_amdgcn_mov_dpp(v, QP_XOR2, 0xF, 0xF, false);
    } else if constexpr (J == 4) {
        // lanes 0-3 and 8-11 of each row read 4 lanes up, the others 4 down
        const int t = __builtin_amdgcn_mov_dpp(v, ROW_SHL4, 0xF, 0x5, false);
        return __builtin_amdgcn_update_dpp(t, v, ROW_SHR4, 0xF, 0xA, false);
    } else if constexpr (J == 8) {
        return __builtin_amdgcn_mov_dpp(v, ROW_ROR8, 0xF, 0xF, false);
    } else if constexpr (J == 16) {
        return __builtin_amdgcn_ds_swizzle(v, 0x401F);    // and 0x1f, or 0, xor 0x10
    } else {
        return __builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ 32u) << 2), v);
    }
}
template <int J>
__device__ __forceinline__ u64_t xor_lane(u64_t v) {
    const int lo = xor_lane<J>((int)(unsigned)v), hi = xor_lane<J>((int)(unsigned)(v >> 32));
    return ((u64_t)(unsigned)hi << 32) | (unsigned)lo;
}

// Number of lanes below this one whose bit is set in m.
__device__ __forceinline__ int lanes_below(u64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

}  // namespace wave
}  // namespace epic
