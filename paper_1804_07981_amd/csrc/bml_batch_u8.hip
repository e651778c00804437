// bml_batch_u8.hip -- instantiates the batched step kernel for the
// byte layout, steps per pass K = 1..MAX_K.
#include "bml_batch.hpp"

namespace bml {

void batch_table_u8(BatchFn *tab)
{
    fill_batch_table<IO_U8, 1>(tab, std::make_integer_sequence<int, MAX_K>{});
}

} // namespace bml
