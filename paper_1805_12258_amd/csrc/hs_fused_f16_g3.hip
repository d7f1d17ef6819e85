// Fused kernels for fp16 FOP storage, H = 13..16.
#define HS_INST_T _Float16
#define HS_INST_NAME f16
#define HS_INST_GROUP 3
#include "hs_fused_inst.h"
