// Recurrence kernels of 5 64-row slot(s) per lane (columns of up to 320 rows).
#define STX_SLOTS 5
#include "inst_body.h"
