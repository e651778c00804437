// bml_pass_u8_lo.hip -- instantiates the streaming step kernel for the
// byte layout, steps per pass K = 1..4 (one translation unit
// per variant group keeps the build parallel).
#include "bml_pass.hpp"

namespace bml {

void pass_table_u8_lo(PassFn *tab)
{
    fill_pass_table<IO_U8, 0, 1>(tab, std::make_integer_sequence<int, 4>{});
}

} // namespace bml
