// The fused log-sum-exp statistic for fp32 FOP storage,
// H = 5..8.
#define HS_INST_T float
#define HS_INST_NAME f32
#define HS_INST_GROUP 1
#define HS_INST_STAT 1
#include "hs_fused_inst.h"
