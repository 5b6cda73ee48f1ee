// Column-kernel instances: element type double, diagnostics false.
#define MAM_INST_T double
#define MAM_INST_DIAG false
#include "mam_instances.hpp"
