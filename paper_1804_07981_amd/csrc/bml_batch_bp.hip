// bml_batch_bp.hip -- instantiates the batched step kernel for the
// bitplane layout, steps per pass K = 1..MAX_K.
#include "bml_batch.hpp"

namespace bml {

void batch_table_bp(BatchFn *tab)
{
    fill_batch_table<IO_BP, 1>(tab, std::make_integer_sequence<int, MAX_K>{});
}

} // namespace bml
