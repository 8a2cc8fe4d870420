// Register-resident 2D-OMP for FP32 at fixed shapes (placeholder: no shapes yet).
#include "sdl_internal.h"

namespace sdl {

template <typename T>
bool omp_fast_supported(int, int, int, int, int) { return false; }

template <typename T>
hipError_t launch_omp_fast(const OmpArgs<T>&, hipStream_t) { return hipErrorInvalidValue; }

template bool omp_fast_supported<float>(int, int, int, int, int);
template bool omp_fast_supported<double>(int, int, int, int, int);
template hipError_t launch_omp_fast<float>(const OmpArgs<float>&, hipStream_t);
template hipError_t launch_omp_fast<double>(const OmpArgs<double>&, hipStream_t);

}  // namespace sdl
