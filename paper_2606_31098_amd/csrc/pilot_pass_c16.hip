// Pass kernels for C = 16 channels (f32 and bf16; G = 4, 8, 16; kernel variants 1 to 10).
#include "pilot_kernels.h"
#include "pilot_pass.inc"
#include "pilot_pass2.inc"
#include "pilot_pass3.inc"
#include "pilot_pass4.inc"

namespace pilot {
PILOT_INSTANTIATE_PASS(16)
}  // namespace pilot
