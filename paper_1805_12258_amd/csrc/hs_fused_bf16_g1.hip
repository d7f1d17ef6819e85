// Fused kernels for bfloat16 FOP storage, H = 5..8.
#define HS_INST_T bf16_t
#define HS_INST_NAME bf16
#define HS_INST_GROUP 1
#include "hs_fused_inst.h"
