// Kernels and launchers for SU(4).
#include "sun_ops_impl.hpp"
SUN_DEFINE_OPS(4)
