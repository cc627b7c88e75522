#define SSGP_REAL double
#include "tu_adj.inc"
