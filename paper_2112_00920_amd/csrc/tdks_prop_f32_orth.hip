// k_propagate instantiations: float, orthogonal cells, real-time step, observation and h application.
#define REAL float
#define NONORTH_FLAG false
#define ITIME_FLAG false
#define LAUNCH_NAME launch_propagate_f32_orth
#include "tdks_prop_dispatch.h"
