// Fused kernels for bfloat16 FOP storage, H = 13..16.
#define HS_INST_T bf16_t
#define HS_INST_NAME bf16
#define HS_INST_GROUP 3
#include "hs_fused_inst.h"
