#define SSGP_REAL float
#include "tu_1d.inc"
