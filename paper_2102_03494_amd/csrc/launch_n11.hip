// Kernel instances and launch wrappers for rings of N = 2^11.
#include "launch.h"

HE_INSTANTIATE_LAUNCHERS(11)
