// Instantiates the fused stage kernel variants for FP32 states of order 8.
#define SBLI_STAGE_TU_TYPE float
#define SBLI_STAGE_TU_R 4
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_F4
#include "stage_variants.h"
