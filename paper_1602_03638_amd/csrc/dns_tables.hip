// Dispatch from a run-time size to the launch table of each precision; the
// tables themselves are compiled per (precision, N) from dns_inst.hip.
#include "dns_ops.hpp"

namespace dns {

#define DNS_DECLARE_TABLES(R)                                  \
    template <> const Ops* ops_table<R, 8>();                  \
    template <> const Ops* ops_table<R, 16>();                 \
    template <> const Ops* ops_table<R, 32>();                 \
    template <> const Ops* ops_table<R, 64>();                 \
    template <> const Ops* ops_table<R, 128>();                \
    template <> const Ops* ops_table<R, 256>();                \
    template <> const Ops* ops_table<R, 512>();                \
    template <> const Ops* ops_table<R, 1024>();
DNS_DECLARE_TABLES(double)
DNS_DECLARE_TABLES(float)
#undef DNS_DECLARE_TABLES

template <typename R> static const Ops* table_for(int N) {
    switch (N) {
        case 8: return ops_table<R, 8>();
        case 16: return ops_table<R, 16>();
        case 32: return ops_table<R, 32>();
        case 64: return ops_table<R, 64>();
        case 128: return ops_table<R, 128>();
        case 256: return ops_table<R, 256>();
        case 512: return ops_table<R, 512>();
        case 1024: return ops_table<R, 1024>();
        default: return nullptr;
    }
}

const Ops* ops_f64(int N) { return table_for<double>(N); }
const Ops* ops_f32(int N) { return table_for<float>(N); }

}  // namespace dns
