// k_f32s.hip -- kernel instantiations for FP32 shifted-deviation storage.
#include "instantiate.hpp"

namespace lbm {
const PrecTable &table_f32s()
{
    static const PrecTable t = make_table<P_F32S>();
    return t;
}
} // namespace lbm
