// bml_block.hip -- instantiates the register-resident tile kernel
// (bml_block.hpp) for both layouts and both update rules it runs.
#include "bml_block.hpp"

namespace bml {

void block_kernels(BlockFn (*fn)[2])
{
    fn[IO_U8][0] = block_kernel<IO_U8, 1>;
    fn[IO_U8][1] = block_kernel<IO_U8, 3>;
    fn[IO_BP][0] = block_kernel<IO_BP, 1>;
    fn[IO_BP][1] = block_kernel<IO_BP, 3>;
}

} // namespace bml
