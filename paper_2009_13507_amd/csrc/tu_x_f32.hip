#define SSGP_REAL float
#define SSGP_REAL_IS_DOUBLE 0
#include "tu_x.inc"
