// Instantiates the fused stage kernel variants for FP64 states of order 2.
#define SBLI_STAGE_TU_TYPE double
#define SBLI_STAGE_TU_R 1
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_D1
#include "stage_variants.h"
