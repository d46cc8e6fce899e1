// k_propagate instantiations: float, non-orthogonal cells, real-time step, observation and h application.
#define REAL float
#define NONORTH_FLAG true
#define ITIME_FLAG false
#define LAUNCH_NAME launch_propagate_f32_nonorth
#include "tdks_prop_dispatch.h"
