// relax_flat.hip -- the relaxation kernel variants that read the flat layout (one sorted departure array per type).
#include "relax.hpp"

namespace eat {

RelaxFn relax_fn_flat(int tpv, int ub, int block, bool goal) { return relax_fn<kKindFlat>(tpv, ub, block, goal); }

}  // namespace eat
