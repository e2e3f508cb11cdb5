// Kernel instantiations: dim = 2, FP64 arithmetic, degrees 1..8.
#include "inst.hpp"
DGW_DEFINE_INST(launchers_d2_f64, 2, double)
