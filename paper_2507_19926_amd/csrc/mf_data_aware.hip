// Data-aware variant: placeholder until the LDS merge kernel lands.
#include "mf_internal.h"

bool mf_da_supports(int, int, int, int) { return false; }
void mf_da_default_tile(int, int, int* tw, int* th) { *tw = *th = 1; }
hipError_t mf_da_launch(const void*, void*, int, int, long long, int, int, int, int, hipStream_t)
{
    return hipErrorNotSupported;
}
