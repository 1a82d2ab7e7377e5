// Instantiates the fused stage kernel variants for FP64 states of order 4.
#define SBLI_STAGE_TU_TYPE double
#define SBLI_STAGE_TU_R 2
#define SBLI_STAGE_TU_LIST SBLI_VARIANTS_D2
#include "stage_variants.h"
