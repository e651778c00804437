// bml_block.hip -- instantiates the register-resident tile kernel
// (bml_block.hpp) for both layouts.
#include "bml_block.hpp"

namespace bml {

void block_kernels(BlockFn *u8, BlockFn *bp)
{
    *u8 = block_kernel<IO_U8>;
    *bp = block_kernel<IO_BP>;
}

} // namespace bml
