// Recurrence kernels of 16 64-row slot(s) per lane (columns of up to 1024 rows).
#define STX_SLOTS 16
#include "inst_body.h"
