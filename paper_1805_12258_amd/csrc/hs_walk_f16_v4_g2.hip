// Strip-walk detection kernels for f16 FOP storage, 4 bins per lane,
// H = 9..12.
#define HS_WALK_T _Float16
#define HS_WALK_NAME f16
#define HS_WALK_V 4
#define HS_WALK_GROUP 2
#include "hs_walk_inst.h"
