// cr_ik_self_ext.hip -- Algorithm 1 with self contact and extensible segments
// (instantiations of the generic IK path, three to six segments).
#include "cr_ik_gen.h"

namespace crk {

CR_IK_GEN_INST(true, true, 3)
CR_IK_GEN_INST(true, true, 4)
CR_IK_GEN_INST(true, true, 5)
CR_IK_GEN_INST(true, true, 6)

}  // namespace crk
