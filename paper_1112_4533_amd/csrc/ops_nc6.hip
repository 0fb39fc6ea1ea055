// Kernels and launchers for SU(6).  Matrix loops stay rolled (see
// SUN_MAT_UNROLL): at this Nc a link matrix does not fit in registers.
#define SUN_MAT_UNROLL _Pragma("unroll 1")
#include "sun_ops_impl.hpp"
SUN_DEFINE_OPS(6)
