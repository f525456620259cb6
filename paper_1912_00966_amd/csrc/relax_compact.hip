// relax_compact.hip -- the relaxation kernel variants that read the hybrid layout's compact cluster headers.
#include "relax.hpp"

namespace eat {

RelaxFn relax_fn_compact(int tpv, int ub, int block, bool goal) { return relax_fn<kKindCompact>(tpv, ub, block, goal); }

}  // namespace eat
