// Pseudo-particle builder (replaced by the full implementation).
#include "common.hpp"
namespace sphmap {
void pseudo_build(Ctx &ctx, PseudoArgs &a, hipStream_t s) {
  (void)ctx; (void)a; (void)s;
  throw Error{SPHMAP_EINVAL, "pseudo-particle builder not available"};
}
}  // namespace sphmap
