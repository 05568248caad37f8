// FFT pass launchers, single precision (the CG operator of the mixed form).
#include "fg_fft_impl.hpp"
namespace fg {
FG_INSTANTIATE_LAUNCHERS(float)
}
