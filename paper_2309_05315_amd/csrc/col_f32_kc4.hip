// Column-kernel instances: element type float, 4 column(s) in flight.
#define MAM_INST_T float
#define MAM_INST_KC 4
#include "mam_instances.hpp"
