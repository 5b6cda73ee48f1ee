// Column-kernel instances: element type double, 4 column(s) in flight.
#define MAM_INST_T double
#define MAM_INST_KC 4
#include "mam_instances.hpp"
