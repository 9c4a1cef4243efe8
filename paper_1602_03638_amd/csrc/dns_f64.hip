// FP64 instantiation of every kernel for N = 8 .. 1024.
#include "dns_impl.hpp"

namespace dns {
const Ops* ops_f64(int N) { return ops_for<double>(N); }
}  // namespace dns
