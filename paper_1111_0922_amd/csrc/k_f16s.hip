// k_f16s.hip -- kernel instantiations for f16s PDF storage.
#include "instantiate.hpp"

namespace lbm {
const PrecTable &table_f16s()
{
    static const PrecTable t = make_table<P_F16S>();
    return t;
}
} // namespace lbm
