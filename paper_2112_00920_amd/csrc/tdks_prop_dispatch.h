// Dispatch of the k_propagate instantiations of one translation unit.  The including
// file defines REAL (float / double), NONORTH_FLAG (non-orthogonal cells: the kernel's
// NONORTH is then 1, or 2 with the mixed derivatives through the LDS intermediate when
// PropArgs::mixt is set), ITIME_FLAG (imaginary-time variant) and LAUNCH_NAME; the split
// lets the variants compile in parallel.
#pragma once
#include "tdks_propagate.h"

namespace tdks {

template <int ZL, int MAXT, int MINW, int SL, bool RAGGED, int NO, bool GC>
static hipError_t launch_gc(const PropArgs &a, int n_items, int block, hipStream_t s) {
    auto kern = k_propagate<REAL, ZL, NO, MAXT, MINW, SL, RAGGED, ITIME_FLAG, GC>;
    const size_t lds = propagate_lds_bytes_inl(sizeof(REAL) == 8, SL == 1, a, block);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

// the global column tables are built for FP64 only (the FP32 tables fit the LDS)
template <int ZL, int MAXT, int MINW, int SL, bool RAGGED, int NO>
static hipError_t launch_no(const PropArgs &a, int n_items, int block, hipStream_t s) {
    if constexpr (sizeof(REAL) == 8 && SL != 1) {
        if (a.gcol) return launch_gc<ZL, MAXT, MINW, SL, RAGGED, NO, true>(a, n_items, block, s);
    }
    if (a.gcol) return hipErrorInvalidValue;
    return launch_gc<ZL, MAXT, MINW, SL, RAGGED, NO, false>(a, n_items, block, s);
}

template <int ZL, int MAXT, int MINW, int SL, bool RAGGED>
static hipError_t launch_zl(const PropArgs &a, int n_items, int block, hipStream_t s) {
    if (!NONORTH_FLAG) return launch_no<ZL, MAXT, MINW, SL, RAGGED, 0>(a, n_items, block, s);
    return a.mixt ? launch_no<ZL, MAXT, MINW, SL, RAGGED, 2>(a, n_items, block, s)
                  : launch_no<ZL, MAXT, MINW, SL, RAGGED, 1>(a, n_items, block, s);
}

template <bool IT>
static hipError_t dispatch(const PropArgs &a, int n_items, int block, int zl, int minw, int sl, int ragged,
                           hipStream_t s) {
// FP64 reads the projector records from global memory only (SL 0); FP32 stages them (1) or
// their CSR pointers (2) in LDS when they fit
#define TDKS_CASE(Z, M, O, RG)                                                                      \
    if (ragged == RG && zl == Z && block <= M && minw == O) {                                       \
        if constexpr (sizeof(REAL) == 8) {                                                          \
            if (sl || a.ptp_lds) return hipErrorInvalidValue;                                       \
            return launch_zl<Z, M, O, 0, RG>(a, n_items, block, s);                                 \
        } else {                                                                                    \
            return sl ? launch_zl<Z, M, O, 1, RG>(a, n_items, block, s)                             \
                      : a.ptp_lds ? launch_zl<Z, M, O, 2, RG>(a, n_items, block, s)                 \
                                  : launch_zl<Z, M, O, 0, RG>(a, n_items, block, s);                \
        }                                                                                           \
    }
#define TDKS_CASE_EVEN(Z, M, O) TDKS_CASE(Z, M, O, false)
#define TDKS_CASE_RAGGED(Z, M, O) TDKS_CASE(Z, M, O, true)
    TDKS_PROPAGATE_CONFIGS(TDKS_CASE_EVEN)
    TDKS_PROPAGATE_RAGGED_CONFIGS(TDKS_CASE_RAGGED)
#undef TDKS_CASE_RAGGED
#undef TDKS_CASE_EVEN
#undef TDKS_CASE
    return hipErrorInvalidValue;
}

hipError_t LAUNCH_NAME(const PropArgs &a, int n_items, int block, int zl, int minw, int sl, int ragged,
                       hipStream_t s) {
    return dispatch<ITIME_FLAG>(a, n_items, block, zl, minw, sl, ragged, s);
}

}  // namespace tdks
