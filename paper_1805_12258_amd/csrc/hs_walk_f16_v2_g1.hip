// Strip-walk detection kernels for f16 FOP storage, 2 bins per lane,
// H = 5..8.
#define HS_WALK_T _Float16
#define HS_WALK_NAME f16
#define HS_WALK_V 2
#define HS_WALK_GROUP 1
#include "hs_walk_inst.h"
