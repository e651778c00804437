// bml_block.hip -- instantiates the register-resident tile kernel
// (bml_block.hpp) for both layouts, both update rules it runs and the
// three tile widths.
#include "bml_block.hpp"

namespace bml {

template <int IO, int MODEL>
static void widths(BlockFn *fn)
{
    fn[0] = block_kernel<IO, MODEL, 32>;
    fn[1] = block_kernel<IO, MODEL, 16>;
    fn[2] = block_kernel<IO, MODEL, 8>;
}

void block_kernels(BlockFn (*fn)[2][3])
{
    widths<IO_U8, 1>(fn[IO_U8][0]);
    widths<IO_U8, 3>(fn[IO_U8][1]);
    widths<IO_BP, 1>(fn[IO_BP][0]);
    widths<IO_BP, 3>(fn[IO_BP][1]);
}

} // namespace bml
