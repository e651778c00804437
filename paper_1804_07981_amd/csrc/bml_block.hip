// bml_block.hip -- instantiates the register-resident tile kernel
// (bml_block.hpp) for both layouts, the update rules and topologies it runs
// and the three tile widths.
#include "bml_block.hpp"

namespace bml {

template <int IO, int MODEL, bool KLEIN>
static void widths(BlockFn *fn)
{
    fn[0] = block_kernel<IO, MODEL, 32, KLEIN>;
    fn[1] = block_kernel<IO, MODEL, 16, KLEIN>;
    fn[2] = block_kernel<IO, MODEL, 8, KLEIN>;
}

void block_kernels(BlockFn (*fn)[3][3])
{
    widths<IO_U8, 1, false>(fn[IO_U8][0]);
    widths<IO_U8, 3, false>(fn[IO_U8][1]);
    widths<IO_U8, 1, true>(fn[IO_U8][2]);
    widths<IO_BP, 1, false>(fn[IO_BP][0]);
    widths<IO_BP, 3, false>(fn[IO_BP][1]);
    widths<IO_BP, 1, true>(fn[IO_BP][2]);
}

} // namespace bml
