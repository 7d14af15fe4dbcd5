// Recurrence kernels of 3 64-row slot(s) per lane (columns of up to 192 rows).
#define STX_SLOTS 3
#include "inst_body.h"
