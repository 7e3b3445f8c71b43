// k_f64.hip -- kernel instantiations for f64 PDF storage.
#include "instantiate.hpp"

namespace lbm {
const PrecTable &table_f64()
{
    static const PrecTable t = make_table<P_F64>();
    return t;
}
} // namespace lbm
