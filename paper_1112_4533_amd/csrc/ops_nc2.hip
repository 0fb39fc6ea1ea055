// Kernels and launchers for SU(2).
#include "sun_ops_impl.hpp"
SUN_DEFINE_OPS(2)
