// pic_dpp.h -- wavefront scans on DPP (GFX9 data-parallel primitives) for gfx950.
#pragma once
#include <hip/hip_runtime.h>

namespace pic {

// ---------------------------------------------------------------------------------------------
// Wavefront segmented inclusive scan on DPP (GFX9 data-parallel primitives): four row shifts
// within rows of 16 lanes, then the row-15 and row-31 broadcasts.  Lanes hold consecutive
// (cell-sorted) particles; a segment starts where the start node differs from the previous lane.
// The per-step "add" predicates depend only on the segment heads, so they are computed once and
// reused for every value.
// ---------------------------------------------------------------------------------------------
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, false);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_r(int v)
{
    return dpp_i<CTRL, ROWMASK>(v);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_r(float v)
{
    return __builtin_bit_cast(float, dpp_i<CTRL, ROWMASK>(__builtin_bit_cast(int, v)));
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_r(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_i<CTRL, ROWMASK>((int)(b & 0xffffffffll));
    const int hi = dpp_i<CTRL, ROWMASK>((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ unsigned seg_masks(bool head)
{
    int f = head ? 1 : 0;
    unsigned m = 0;
    int fu;
    fu = dpp_i<kRowShr1, 0xf>(f);    if (!f) m |= 1u;  f |= fu;
    fu = dpp_i<kRowShr2, 0xf>(f);    if (!f) m |= 2u;  f |= fu;
    fu = dpp_i<kRowShr4, 0xf>(f);    if (!f) m |= 4u;  f |= fu;
    fu = dpp_i<kRowShr8, 0xf>(f);    if (!f) m |= 8u;  f |= fu;
    fu = dpp_i<kRowBcast15, 0xa>(f); if (!f) m |= 16u; f |= fu;
    fu = dpp_i<kRowBcast31, 0xc>(f); if (!f) m |= 32u;
    return m;
}

template <typename R>
__device__ __forceinline__ R seg_scan(R v, unsigned m)
{
    R t;
    t = dpp_r<kRowShr1, 0xf>(v);    if (m & 1u) v += t;
    t = dpp_r<kRowShr2, 0xf>(v);    if (m & 2u) v += t;
    t = dpp_r<kRowShr4, 0xf>(v);    if (m & 4u) v += t;
    t = dpp_r<kRowShr8, 0xf>(v);    if (m & 8u) v += t;
    t = dpp_r<kRowBcast15, 0xa>(v); if (m & 16u) v += t;
    t = dpp_r<kRowBcast31, 0xc>(v); if (m & 32u) v += t;
    return v;
}

// Segmented inclusive scan of N values at once over the first STEPS DPP steps (STEPS <= 6: the
// scan spans groups of 2^STEPS lanes).  Step k is applied to every value before step k + 1, so
// the DPP reads of one value follow the writes of the others and need no wait states.
template <int STEPS, int N, typename R>
__device__ __forceinline__ void seg_scan_n(R (&v)[N], unsigned m)
{
    R t[N];
#define PIC_SCAN_STEP(K, CTRL, ROWMASK)                                                \
    if (STEPS > K) {                                                                   \
        _Pragma("unroll") for (int q = 0; q < N; ++q) t[q] = dpp_r<CTRL, ROWMASK>(v[q]); \
        _Pragma("unroll") for (int q = 0; q < N; ++q) if (m & (1u << K)) v[q] += t[q];  \
    }
    PIC_SCAN_STEP(0, kRowShr1, 0xf)
    PIC_SCAN_STEP(1, kRowShr2, 0xf)
    PIC_SCAN_STEP(2, kRowShr4, 0xf)
    PIC_SCAN_STEP(3, kRowShr8, 0xf)
    PIC_SCAN_STEP(4, kRowBcast15, 0xa)
    PIC_SCAN_STEP(5, kRowBcast31, 0xc)
#undef PIC_SCAN_STEP
}

// Step masks of seg_masks for the first STEPS steps only.
template <int STEPS>
__device__ __forceinline__ unsigned seg_masks_n(bool head)
{
    int f = head ? 1 : 0;
    unsigned m = 0;
    int fu;
    if (STEPS > 0) { fu = dpp_i<kRowShr1, 0xf>(f);    if (!f) m |= 1u;  f |= fu; }
    if (STEPS > 1) { fu = dpp_i<kRowShr2, 0xf>(f);    if (!f) m |= 2u;  f |= fu; }
    if (STEPS > 2) { fu = dpp_i<kRowShr4, 0xf>(f);    if (!f) m |= 4u;  f |= fu; }
    if (STEPS > 3) { fu = dpp_i<kRowShr8, 0xf>(f);    if (!f) m |= 8u;  f |= fu; }
    if (STEPS > 4) { fu = dpp_i<kRowBcast15, 0xa>(f); if (!f) m |= 16u; f |= fu; }
    if (STEPS > 5) { if (!f) m |= 32u; }
    return m;
}

// Plain inclusive scan over the whole wavefront (one segment starting at lane 0).
__device__ __forceinline__ unsigned scan_masks(int lane) { return seg_masks(lane == 0); }

}  // namespace pic
