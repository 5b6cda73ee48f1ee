// Column-kernel instances: element type float, diagnostics instances.
#define MAM_INST_T float
#define MAM_INST_KC 0
#include "mam_instances.hpp"
