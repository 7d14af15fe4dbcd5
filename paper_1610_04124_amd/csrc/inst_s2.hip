// Recurrence kernels of 2 64-row slot(s) per lane (columns of up to 128 rows).
#define STX_SLOTS 2
#include "inst_body.h"
