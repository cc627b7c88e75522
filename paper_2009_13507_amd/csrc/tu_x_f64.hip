#define SSGP_REAL double
#include "tu_x.inc"
