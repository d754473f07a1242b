// Row-pass instantiations: C_Q in double, p / 16 = 1 mod 4.
#define HIKF_RP_TQ double
#define HIKF_RP_SEL 1
#include "rowpass.h"
