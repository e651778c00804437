// bml_resident_u8.hip -- instantiates the register-resident batched kernel
// (bml_resident.hpp) for uint8 cells (one translation unit per layout, so
// the two compile in parallel).
#include "bml_resident.hpp"

namespace bml {

ResidentFn resident_kernel_u8()
{
    return resident_kernel<IO_U8>;
}

} // namespace bml
