// AMR trees: not yet provided.
#include "tree_amr.h"

namespace cd {
int amr_build(cd_tree*, const int64_t*, const int32_t* const*, const float*, int64_t, hipStream_t) {
    set_error("cd_build_tree: AMR trees are not provided by this build");
    return CD_EUNSUPPORTED;
}
int amr_update(cd_tree*, const float*, hipStream_t) {
    set_error("cd_tree_update: AMR trees are not provided by this build");
    return CD_EUNSUPPORTED;
}
int amr_leaf_coords(const cd_tree*, int8_t*, int32_t*) { return CD_EUNSUPPORTED; }
int amr_columns(cd_tree*, const cd_weights*, float*, float*, float, hipStream_t) { return CD_EUNSUPPORTED; }
}  // namespace cd
