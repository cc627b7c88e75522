#define SSGP_REAL float
#include "tu_batch.inc"
