// AMR part of the tree (levels finer than the base grid).
#pragma once

#include "cd_internal.h"

namespace cd {
int amr_build(cd_tree* t, const int64_t* n_octs, const int32_t* const* oct_parents, const float* leaf_n_dev,
              int64_t n_leaf, hipStream_t s);
int amr_update(cd_tree* t, const float* leaf_n_dev, hipStream_t s);
int amr_leaf_coords(const cd_tree* t, int8_t* level, int32_t* ijk);
int amr_columns(cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale, hipStream_t s);
void amr_free(cd_tree* t);
int build_dense_below(cd_tree* t, int top, hipStream_t s);
int alloc_dense_levels(cd_tree* t, int top, hipStream_t s);
}  // namespace cd
