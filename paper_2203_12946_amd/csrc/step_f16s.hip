// Instantiation of the step kernel for half-precision deviations f - w (one translation unit
// per storage type, so that the library's sources compile in parallel).
#include "step_kernel.hpp"

namespace eselbm {

hipError_t launch_step_f16s(int D, int mode, bool diag, const StepArgs &a, hipStream_t s)
{
    return launch_step_storage<_Float16>(D, mode, diag, a, s);
}

}  // namespace eselbm
