// cr_ik_ext.hip -- Algorithm 1 for robots with extensible segments (instantiations
// of the generic IK path, one to six segments, FP32 and FP64 stage 1).
#include "cr_ik_gen.h"

namespace crk {

CR_IK_GEN_INST(true, false, 1)
CR_IK_GEN_INST(true, false, 2)
CR_IK_GEN_INST(true, false, 3)
CR_IK_GEN_INST(true, false, 4)
CR_IK_GEN_INST(true, false, 5)
CR_IK_GEN_INST(true, false, 6)

}  // namespace crk
