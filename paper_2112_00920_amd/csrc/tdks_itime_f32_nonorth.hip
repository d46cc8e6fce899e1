// k_propagate instantiations: float, non-orthogonal cells, imaginary-time Taylor step.
#define REAL float
#define NONORTH_FLAG true
#define ITIME_FLAG true
#define LAUNCH_NAME launch_itime_f32_nonorth
#include "tdks_prop_dispatch.h"
