// bml_pass_inst.hip -- instantiates the streaming step kernel for one layout,
// column mode / range of K and topology, chosen by the build:
//   BML_INST_IO (IO_U8 / IO_BP), BML_INST_ROW (0 tile, 1 or 2 words per lane
//   in row mode), BML_INST_TOPO (TOPO_TORUS / TOPO_KLEIN), BML_INST_MODEL (1
//   or 2), BML_INST_KLO and BML_INST_KN (K = KLO .. KLO + KN - 1),
//   BML_INST_NAME (the table function).
#include "bml_pass.hpp"

namespace bml {

void BML_INST_NAME(PassFn *tab)
{
    fill_pass_table<BML_INST_IO, BML_INST_ROW, BML_INST_TOPO, BML_INST_MODEL, BML_INST_KLO>(
        tab, std::make_integer_sequence<int, BML_INST_KN>{});
}

} // namespace bml
