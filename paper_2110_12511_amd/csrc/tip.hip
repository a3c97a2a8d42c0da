#include "pbng_internal.h"
namespace pbng {
void tip_decompose(Ctx &, const DevGraph &, int, const pbng_opts &, u64 *) {
    throw Error(PBNG_E_UNSUPPORTED, "tip decomposition not built yet");
}
}  // namespace pbng
