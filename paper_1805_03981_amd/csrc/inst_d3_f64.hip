// Kernel instantiations: dim = 3, FP64 arithmetic, degrees 1..8.
#include "inst.hpp"
DGW_DEFINE_INST(launchers_d3_f64, 3, double)
