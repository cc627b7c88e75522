#define SSGP_REAL double
#define SSGP_REAL_IS_DOUBLE 1
#include "tu_x.inc"
