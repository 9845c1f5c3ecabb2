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

// FP32 form of seg_scan_n, on groups of 16 lanes (one DPP row; STEPS <= 4), for the N = 5, 8 and
// 12 deposit values of 1D, 2D and 3D: each step adds the row-shifted value times a per-lane 0/1
// factor with one v_fmac_f32 that takes its first operand through DPP (v + 1 * t rounds as v + t;
// v + 0 * t is v), in place of a shift, an add and a select.  Written as assembly because the
// compiler does not fold a DPP move into an FMA.  Source lanes outside the row are disabled by the
// row shift (no bound_ctrl), so those lanes keep v.  A VALU write followed by a DPP read of the same
// register needs two wait states on this architecture and the compiler cannot see into the asm, so
// each step is one asm statement that starts with s_nop 1 (nothing can be scheduled between the
// wait and the reads), and the last step ends with one.
#define PIC_FM(i, f, sh) "v_fmac_f32_dpp %" #i ", %" #i ", %" #f " row_shr:" #sh " row_mask:0xf bank_mask:0xf\n\t"
#define PIC_FM5(f, sh) PIC_FM(0, f, sh) PIC_FM(1, f, sh) PIC_FM(2, f, sh) PIC_FM(3, f, sh) PIC_FM(4, f, sh)
#define PIC_FM8(f, sh) PIC_FM5(f, sh) PIC_FM(5, f, sh) PIC_FM(6, f, sh) PIC_FM(7, f, sh)
#define PIC_FM12(f, sh) PIC_FM8(f, sh) PIC_FM(8, f, sh) PIC_FM(9, f, sh) PIC_FM(10, f, sh) PIC_FM(11, f, sh)
#define PIC_V5 "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4])
#define PIC_V8 PIC_V5, "+v"(v[5]), "+v"(v[6]), "+v"(v[7])
#define PIC_V12 PIC_V8, "+v"(v[8]), "+v"(v[9]), "+v"(v[10]), "+v"(v[11])

template <int N, int SH, bool LAST>
__device__ __forceinline__ void fmac_step(float (&v)[N], float f)
{
    static_assert(N == 5 || N == 8 || N == 12, "deposit value counts of 1D, 2D, 3D");
#define PIC_STEP_ASM(NN, sh)                                                                        \
    if constexpr (N == NN && SH == sh) {                                                            \
        if constexpr (LAST)                                                                         \
            asm volatile("s_nop 1\n\t" PIC_FM##NN(NN, sh) "s_nop 1" : PIC_V##NN : "v"(f));          \
        else                                                                                        \
            asm volatile("s_nop 1\n\t" PIC_FM##NN(NN, sh) : PIC_V##NN : "v"(f));                    \
    }
    PIC_STEP_ASM(5, 1) PIC_STEP_ASM(5, 2) PIC_STEP_ASM(5, 4) PIC_STEP_ASM(5, 8)
    PIC_STEP_ASM(8, 1) PIC_STEP_ASM(8, 2) PIC_STEP_ASM(8, 4) PIC_STEP_ASM(8, 8)
    PIC_STEP_ASM(12, 1) PIC_STEP_ASM(12, 2) PIC_STEP_ASM(12, 4) PIC_STEP_ASM(12, 8)
#undef PIC_STEP_ASM
}
#undef PIC_FM
#undef PIC_FM5
#undef PIC_FM8
#undef PIC_FM12
#undef PIC_V5
#undef PIC_V8
#undef PIC_V12

template <int STEPS, int N>
__device__ __forceinline__ void seg_scan_n(float (&v)[N], unsigned m)
{
    static_assert(STEPS >= 1 && STEPS <= 4, "row shifts only");
    const float f0 = (m & 1u) ? 1.0f : 0.0f, f1 = (m & 2u) ? 1.0f : 0.0f;
    const float f2 = (m & 4u) ? 1.0f : 0.0f, f3 = (m & 8u) ? 1.0f : 0.0f;
    fmac_step<N, 1, STEPS == 1>(v, f0);
    if constexpr (STEPS > 1) fmac_step<N, 2, STEPS == 2>(v, f1);
    if constexpr (STEPS > 2) fmac_step<N, 4, STEPS == 3>(v, f2);
    if constexpr (STEPS > 3) fmac_step<N, 8, true>(v, f3);
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
