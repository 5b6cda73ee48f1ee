// Column-kernel instances: element type float, 2 column(s) in flight.
#define MAM_INST_T float
#define MAM_INST_KC 2
#include "mam_instances.hpp"
