// Kernels and launchers for SU(3).
#include "sun_ops_impl.hpp"
SUN_DEFINE_OPS(3)
