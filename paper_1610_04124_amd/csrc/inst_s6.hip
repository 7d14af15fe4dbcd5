// Recurrence kernels of 6 64-row slot(s) per lane (columns of up to 384 rows).
#define STX_SLOTS 6
#include "inst_body.h"
