// Recurrence kernels of 1 64-row slot(s) per lane (columns of up to 64 rows).
#define STX_SLOTS 1
#include "inst_body.h"
