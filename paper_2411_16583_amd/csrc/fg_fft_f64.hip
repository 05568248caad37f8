// FFT pass launchers, double precision.
#include "fg_fft_impl.hpp"
namespace fg {
FG_INSTANTIATE_LAUNCHERS(double)
}
