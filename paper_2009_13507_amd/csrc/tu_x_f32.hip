#define SSGP_REAL float
#include "tu_x.inc"
