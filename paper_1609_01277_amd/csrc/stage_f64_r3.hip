// Instantiates the fused stage kernel variants for FP64 states of order 6.
#define SBLI_STAGE_TU_TYPE double
#define SBLI_STAGE_TU_R 3
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_D3
#include "stage_variants.h"
