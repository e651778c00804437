// bml_resident.hip -- instantiates the register-resident batched kernel
// (bml_resident.hpp) for both layouts.
#include "bml_resident.hpp"

namespace bml {

void resident_kernels(ResidentFn *u8, ResidentFn *bp)
{
    *u8 = resident_kernel<IO_U8>;
    *bp = resident_kernel<IO_BP>;
}

} // namespace bml
