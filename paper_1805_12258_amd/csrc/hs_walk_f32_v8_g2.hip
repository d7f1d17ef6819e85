// Strip-walk detection kernels for f32 FOP storage, 8 bins per lane,
// H = 9..12.
#define HS_WALK_T float
#define HS_WALK_NAME f32
#define HS_WALK_V 8
#define HS_WALK_GROUP 2
#include "hs_walk_inst.h"
