// cr_ik_self.hip -- Algorithm 1 with self contact between non-adjacent segments
// (eq. 10; instantiations of the generic IK path, three to six segments).
#include "cr_ik_gen.h"

namespace crk {

CR_IK_GEN_INST(false, true, 3)
CR_IK_GEN_INST(false, true, 4)
CR_IK_GEN_INST(false, true, 5)
CR_IK_GEN_INST(false, true, 6)

}  // namespace crk
