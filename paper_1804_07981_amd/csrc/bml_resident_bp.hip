// bml_resident_bp.hip -- instantiates the register-resident batched kernel
// (bml_resident.hpp) for bitplane state (one translation unit per layout,
// so the two compile in parallel).
#include "bml_resident.hpp"

namespace bml {

ResidentFn resident_kernel_bp()
{
    return resident_kernel<IO_BP>;
}

} // namespace bml
