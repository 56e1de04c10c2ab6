// Kernel instances and launch wrappers for rings of N = 2^13.
#include "launch.h"

HE_INSTANTIATE_LAUNCHERS(13)
