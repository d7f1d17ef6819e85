// Strip-walk detection kernels for f32 FOP storage, 2 bins per lane,
// H = 13..16.
#define HS_WALK_T float
#define HS_WALK_NAME f32
#define HS_WALK_V 2
#define HS_WALK_GROUP 3
#include "hs_walk_inst.h"
