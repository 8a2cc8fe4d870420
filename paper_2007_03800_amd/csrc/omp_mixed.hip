// SDL_MIXED_BF16 sparse coding (placeholder until the kernel lands).
#include "sdl_internal.h"

namespace sdl {
bool omp_mixed_supported(int, int, int, int, int) { return false; }
hipError_t launch_omp_mixed(const OmpArgs<float>&, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace sdl
