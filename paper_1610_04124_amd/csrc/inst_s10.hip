// Recurrence kernels of 10 64-row slot(s) per lane (columns of up to 640 rows).
#define STX_SLOTS 10
#include "inst_body.h"
