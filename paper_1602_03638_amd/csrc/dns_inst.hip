// Kernels and launch table of one (real type, N) pair: the build compiles
// this file once per pair with -DDNS_INST_REAL=<double|float> -DDNS_INST_N=<N>.
#include "dns_impl.hpp"
