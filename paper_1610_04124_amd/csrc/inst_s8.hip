// Recurrence kernels of 8 64-row slot(s) per lane (columns of up to 512 rows).
#define STX_SLOTS 8
#include "inst_body.h"
