// k_propagate instantiations: double, orthogonal cells, imaginary-time Taylor step.
#define REAL double
#define NONORTH_FLAG false
#define ITIME_FLAG true
#define LAUNCH_NAME launch_itime_f64_orth
#include "tdks_prop_dispatch.h"
