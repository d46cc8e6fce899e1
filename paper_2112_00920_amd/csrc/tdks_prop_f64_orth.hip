// k_propagate instantiations: double, orthogonal cells, real-time step, observation and h application.
#define REAL double
#define NONORTH_FLAG false
#define ITIME_FLAG false
#define LAUNCH_NAME launch_propagate_f64_orth
#include "tdks_prop_dispatch.h"
