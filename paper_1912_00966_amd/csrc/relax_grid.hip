// relax_grid.hip -- the relaxation kernel variants that read the hybrid layout's header grid.
#include "relax.hpp"

namespace eat {

RelaxFn relax_fn_grid(int tpv, int ub, int block, bool goal) { return relax_fn<kKindGrid>(tpv, ub, block, goal); }

}  // namespace eat
