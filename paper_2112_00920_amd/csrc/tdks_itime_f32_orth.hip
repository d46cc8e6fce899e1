// k_propagate instantiations: float, orthogonal cells, imaginary-time Taylor step.
#define REAL float
#define NONORTH_FLAG false
#define ITIME_FLAG true
#define LAUNCH_NAME launch_itime_f32_orth
#include "tdks_prop_dispatch.h"
