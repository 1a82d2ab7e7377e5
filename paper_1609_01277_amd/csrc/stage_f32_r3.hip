// Instantiates the fused stage kernel variants for FP32 states of order 6.
#define SBLI_STAGE_TU_TYPE float
#define SBLI_STAGE_TU_R 3
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_F3
#include "stage_variants.h"
