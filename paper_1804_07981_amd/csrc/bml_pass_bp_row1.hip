// bml_pass_bp_row1.hip -- instantiates the streaming step kernel in row
// mode for the bitplane layout at N = 2048 (one word per lane), K = 1..8.
#include "bml_pass.hpp"

namespace bml {

void pass_table_bp_row1(PassFn *tab)
{
    fill_pass_table<IO_BP, 1, 1>(tab, std::make_integer_sequence<int, MAX_K>{});
}

} // namespace bml
