#define SSGP_REAL float
#include "tu_adj.inc"
