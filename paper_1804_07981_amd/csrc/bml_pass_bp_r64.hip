// bml_pass_bp_r64.hip -- instantiates the step kernel for the
// bitplane layout with 64-row wavefront tiles, one kernel per
// steps-per-pass K = 1..MAX_K (one translation unit per variant keeps the
// build parallel).
#include "bml_pass.hpp"

namespace bml {

void pass_table_bp_r64(PassFn *tab)
{
    fill_pass_table<IO_BP, 64>(tab, std::make_integer_sequence<int, MAX_K>{});
}

} // namespace bml
