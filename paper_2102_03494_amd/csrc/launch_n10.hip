// Kernel instances and launch wrappers for rings of N = 2^10.
#include "launch.h"

HE_INSTANTIATE_LAUNCHERS(10)
