// Entry points whose kernels are not built yet: they validate nothing and
// report TGEMM_NOT_SUPPORTED so that callers fail loudly.
#include "../../include/tgemm.h"

extern "C" {

int tgemm_batched(int64_t, const int64_t*, const int64_t*, const int64_t*, const float*,
                  const void* const*, const int64_t*, const void* const*, const int64_t*,
                  const float*, float* const*, const int64_t*, int, void*)
{
    return TGEMM_NOT_SUPPORTED;
}


void tgemm_shutdown(void) {}

}
