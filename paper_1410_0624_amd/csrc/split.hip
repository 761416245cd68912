// Split-precision (hi + lo) weight banks for the MFMA sweep: not yet provided.
#include "cd_internal.h"

namespace cd {
int upload_split_banks(cd_weights* w, hipStream_t) {
    (void)w;
    set_error("cd_precompute_weights: split precision is not provided by this build");
    return CD_EUNSUPPORTED;
}
void free_split_banks(cd_weights*) {}
}  // namespace cd
