// Row-pass instantiations: C_Q in double, p / 16 = 2 mod 4.
#define HIKF_RP_TQ double
#define HIKF_RP_SEL 2
#include "rowpass.h"
