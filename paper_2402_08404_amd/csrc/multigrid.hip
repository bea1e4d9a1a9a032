// multigrid.hip -- multigrid-preconditioned and mixed-precision CG (pending).
#include "pic_internal.hpp"

namespace pic {

size_t mg_bytes(const pic_config*) { return 0; }
int mg_setup(pic_ctx*) { return -3; }

int mgcg_solve(pic_ctx*, double*, double, const int64_t*, int, double, int, pic_solve_info*) { return -3; }

int mixed_solve(pic_ctx*, double*, double, const int64_t*, int, double, int, pic_solve_info*) { return -3; }

}  // namespace pic
