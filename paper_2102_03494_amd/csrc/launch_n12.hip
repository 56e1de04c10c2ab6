// Kernel instances and launch wrappers for rings of N = 2^12.
#include "launch.h"

HE_INSTANTIATE_LAUNCHERS(12)
