// Column-kernel instances: element type double, 2 column(s) in flight.
#define MAM_INST_T double
#define MAM_INST_KC 2
#include "mam_instances.hpp"
