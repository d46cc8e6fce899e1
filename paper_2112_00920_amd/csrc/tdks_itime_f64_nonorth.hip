// k_propagate instantiations: double, non-orthogonal cells, imaginary-time Taylor step.
#define REAL double
#define NONORTH_FLAG true
#define ITIME_FLAG true
#define LAUNCH_NAME launch_itime_f64_nonorth
#include "tdks_prop_dispatch.h"
