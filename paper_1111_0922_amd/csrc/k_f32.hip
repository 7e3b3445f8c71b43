// k_f32.hip -- kernel instantiations for f32 PDF storage.
#include "instantiate.hpp"

namespace lbm {
const PrecTable &table_f32()
{
    static const PrecTable t = make_table<P_F32>();
    return t;
}
} // namespace lbm
