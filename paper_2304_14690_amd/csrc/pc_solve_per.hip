// Transform launchers of periodic axes: the packed real DFT variant of the
// line-transform kernels (see pc_transform.h), compiled apart from the
// cosine-transform variant so that the two build in parallel.
#include "pc_transform.h"

namespace pc {
PC_RAD_COMBOS(PC_RAD_INST_PER)
}  // namespace pc
