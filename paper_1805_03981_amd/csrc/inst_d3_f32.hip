// Kernel instantiations: dim = 3, FP32-split arithmetic, degrees 1..8.
#include "inst.hpp"
DGW_DEFINE_INST(launchers_d3_f32, 3, float)
