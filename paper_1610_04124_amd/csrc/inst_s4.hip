// Recurrence kernels of 4 64-row slot(s) per lane (columns of up to 256 rows).
#define STX_SLOTS 4
#include "inst_body.h"
