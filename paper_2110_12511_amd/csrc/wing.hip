#include "pbng_internal.h"
namespace pbng {
void wing_decompose(Ctx &, const DevGraph &, const pbng_opts &, u64 *) {
    throw Error(PBNG_E_UNSUPPORTED, "wing decomposition not built yet");
}
}  // namespace pbng
