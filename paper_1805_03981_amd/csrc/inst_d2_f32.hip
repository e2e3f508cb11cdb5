// Kernel instantiations: dim = 2, FP32-split arithmetic, degrees 1..8.
#include "inst.hpp"
DGW_DEFINE_INST(launchers_d2_f32, 2, float)
