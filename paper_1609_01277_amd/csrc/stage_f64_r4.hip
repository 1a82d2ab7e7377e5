// Instantiates the fused stage kernel variants for FP64 states of order 8.
#define SBLI_STAGE_TU_TYPE double
#define SBLI_STAGE_TU_R 4
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_D4
#include "stage_variants.h"
