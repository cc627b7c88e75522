#define SSGP_REAL double
#include "tu_batch.inc"
