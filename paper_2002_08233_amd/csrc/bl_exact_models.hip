// The exact-mode kernels instantiated for (a, r) energy models other than
// (2, -1) (Sec. 2.2): the same source as bl_exact.hip, compiled on its own
// so that the (2, -1) kernels keep their code object to themselves.  Only
// exact_run_model and exact_forces_model are defined here.
#define BL_EXACT_MODELS_TU
#include "bl_exact.hip"
