#define REAL double
#define NONORTH_FLAG false
#define LAUNCH_NAME launch_propagate_f64_orth
// Instantiations of k_propagate for one arithmetic type and cell kind (split so the
// four variants compile in parallel).
#include "tdks_propagate.h"

namespace tdks {

template <int ZL, int MAXT, int MINW, bool SL, bool RAGGED>
static hipError_t launch_zl(const PropArgs &a, int n_items, int block, hipStream_t s) {
    auto kern = k_propagate<REAL, ZL, NONORTH_FLAG, MAXT, MINW, SL, RAGGED>;
    const size_t lds = propagate_lds_bytes_inl(sizeof(REAL) == 8, SL, a, block);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t LAUNCH_NAME(const PropArgs &a, int n_items, int block, int zl, int minw, int sl, int ragged,
                       hipStream_t s) {
    if (sl) return hipErrorInvalidValue;  // FP64 tables stay in global memory
#define TDKS_CASE(Z, M, O) \
    if (!ragged && zl == Z && block <= M && minw == O) return launch_zl<Z, M, O, false, false>(a, n_items, block, s);
    TDKS_PROPAGATE_CONFIGS(TDKS_CASE)
#undef TDKS_CASE
#define TDKS_CASE(Z, M, O) \
    if (ragged && zl == Z && block <= M && minw == O) return launch_zl<Z, M, O, false, true>(a, n_items, block, s);
    TDKS_PROPAGATE_RAGGED_CONFIGS(TDKS_CASE)
#undef TDKS_CASE
    return hipErrorInvalidValue;
}

}  // namespace tdks
