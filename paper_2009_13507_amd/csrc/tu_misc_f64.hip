#define SSGP_REAL double
#include "tu_misc.inc"
