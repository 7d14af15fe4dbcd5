// Recurrence kernels of 14 64-row slot(s) per lane (columns of up to 896 rows).
#define STX_SLOTS 14
#include "inst_body.h"
