// The fused log-sum-exp statistic for fp32 FOP storage,
// H = 1..4.
#define HS_INST_T float
#define HS_INST_NAME f32
#define HS_INST_GROUP 0
#define HS_INST_STAT 1
#include "hs_fused_inst.h"
