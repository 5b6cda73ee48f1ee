// Column-kernel instances: element type double, 1 column(s) in flight.
#define MAM_INST_T double
#define MAM_INST_KC 1
#include "mam_instances.hpp"
