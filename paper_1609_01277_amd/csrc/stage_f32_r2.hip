// Instantiates the fused stage kernel variants for FP32 states of order 4.
#define SBLI_STAGE_TU_TYPE float
#define SBLI_STAGE_TU_R 2
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_F2
#include "stage_variants.h"
