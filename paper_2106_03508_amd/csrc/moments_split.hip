// Split-precision moment build (bf16 hi/lo products on MFMA).
#include "agf2_internal.h"

namespace agf2 {

void build_moments_split(Handle& h, int N, int Q, const double* L, int npole, int nocc,
                         const double* e, const double* u, double* m0o, double* m1o,
                         double* m0v, double* m1v) {
  (void)h; (void)N; (void)Q; (void)L; (void)npole; (void)nocc; (void)e; (void)u;
  (void)m0o; (void)m1o; (void)m0v; (void)m1v;
  throw Error{AGF2_ERR_ARG, "AGF2_SPLIT_BF16 is not available in this build"};
}

}  // namespace agf2
