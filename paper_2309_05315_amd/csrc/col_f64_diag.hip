// Column-kernel instances: element type double, diagnostics instances.
#define MAM_INST_T double
#define MAM_INST_KC 0
#include "mam_instances.hpp"
