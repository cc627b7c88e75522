#define SSGP_REAL float
#include "tu_misc.inc"
