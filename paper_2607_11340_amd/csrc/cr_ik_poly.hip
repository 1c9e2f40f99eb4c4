// cr_ik_poly.hip -- Algorithm 1 among convex polytopes (obstacles in half-space
// form, eq. 10 with their signed distance; instantiations of the generic IK path,
// one to six segments, FP32 and FP64 stage 1).
#include "cr_ik_gen.h"

namespace crk {

CR_IK_GEN_INST_POLY(1)
CR_IK_GEN_INST_POLY(2)
CR_IK_GEN_INST_POLY(3)
CR_IK_GEN_INST_POLY(4)
CR_IK_GEN_INST_POLY(5)
CR_IK_GEN_INST_POLY(6)

}  // namespace crk
