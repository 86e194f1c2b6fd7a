// Score equations (eq. gradient; Algorithm 1) on top of the factorizations.
#include "rsf.h"

extern "C" rsf_status rsf_grad(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* g,
                               rsf_grad_info* info, void* stream) {
  (void)f; (void)d_z; (void)eps_peel; (void)seed; (void)g; (void)info; (void)stream;
  return RSF_E_INVALID;
}
