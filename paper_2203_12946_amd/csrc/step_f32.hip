// Instantiation of the step kernel for single-precision populations (one translation unit
// per storage type, so that the library's sources compile in parallel).
#include "step_kernel.hpp"

namespace eselbm {

hipError_t launch_step_f32(int D, int mode, bool diag, const StepArgs &a, hipStream_t s)
{
    return launch_step_storage<float>(D, mode, diag, a, s);
}

}  // namespace eselbm
