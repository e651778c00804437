// bml_pass_bp_hi.hip -- instantiates the streaming step kernel for the
// bitplane layout, steps per pass K = 5..8 (one translation unit
// per variant group keeps the build parallel).
#include "bml_pass.hpp"

namespace bml {

void pass_table_bp_hi(PassFn *tab)
{
    fill_pass_table<IO_BP, 0, 5>(tab, std::make_integer_sequence<int, 4>{});
}

} // namespace bml
