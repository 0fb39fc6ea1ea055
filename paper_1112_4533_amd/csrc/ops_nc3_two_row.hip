// Kernels and launchers for SU(3) with two stored rows (12 reals per link).
#include "sun_ops_impl.hpp"
SUN_DEFINE_OPS_TWO_ROW()
