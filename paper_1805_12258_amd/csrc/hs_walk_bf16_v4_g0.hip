// Strip-walk detection kernels for bf16 FOP storage, 4 bins per lane,
// H = 1..4.
#define HS_WALK_T walk::bf16
#define HS_WALK_NAME bf16
#define HS_WALK_V 4
#define HS_WALK_GROUP 0
#include "hs_walk_inst.h"
