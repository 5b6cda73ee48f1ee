// Column-kernel instances: element type double, diagnostics true.
#define MAM_INST_T double
#define MAM_INST_DIAG true
#include "mam_instances.hpp"
