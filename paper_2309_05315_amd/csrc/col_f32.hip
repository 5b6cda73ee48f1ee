// Column-kernel instances: element type float, diagnostics false.
#define MAM_INST_T float
#define MAM_INST_DIAG false
#include "mam_instances.hpp"
