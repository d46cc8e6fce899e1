// k_propagate instantiations: double, non-orthogonal cells, real-time step, observation and h application.
#define REAL double
#define NONORTH_FLAG true
#define ITIME_FLAG false
#define LAUNCH_NAME launch_propagate_f64_nonorth
#include "tdks_prop_dispatch.h"
