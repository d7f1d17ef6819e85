// Fused kernels for fp16 FOP storage, H = 9..12.
#define HS_INST_T _Float16
#define HS_INST_NAME f16
#define HS_INST_GROUP 2
#include "hs_fused_inst.h"
