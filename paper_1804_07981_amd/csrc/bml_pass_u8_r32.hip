// bml_pass_u8_r32.hip -- instantiates the step kernel for the
// byte layout with 32-row wavefront tiles, one kernel per
// steps-per-pass K = 1..MAX_K (one translation unit per variant keeps the
// build parallel).
#include "bml_pass.hpp"

namespace bml {

void pass_table_u8_r32(PassFn *tab)
{
    fill_pass_table<IO_U8, 32>(tab, std::make_integer_sequence<int, MAX_K>{});
}

} // namespace bml
