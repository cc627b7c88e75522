#define SSGP_REAL double
#include "tu_1d.inc"
