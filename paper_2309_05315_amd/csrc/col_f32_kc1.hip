// Column-kernel instances: element type float, 1 column(s) in flight.
#define MAM_INST_T float
#define MAM_INST_KC 1
#include "mam_instances.hpp"
