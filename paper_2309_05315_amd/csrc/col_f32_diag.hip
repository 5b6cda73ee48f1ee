// Column-kernel instances: element type float, diagnostics true.
#define MAM_INST_T float
#define MAM_INST_DIAG true
#include "mam_instances.hpp"
