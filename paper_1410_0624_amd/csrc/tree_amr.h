// AMR part of the tree (levels finer than the base grid).
#pragma once

#include "cd_internal.h"

namespace cd {

// Device view of an adaptive tree's densities: dense padded levels 0..B and,
// above B, per-level oct densities behind dense maps from the level-(l-1)
// cells to their oct (or -1).
struct AmrLookupView {
    const float* lev[CD_MAX_LEVEL + 1];       // padded dense levels 0..B
    const int32_t* octidx[CD_MAX_LEVEL + 1];  // [l > B] over the level-(l-1) grid
    const float* den[CD_MAX_LEVEL + 1];       // [l > B] oct densities of level l
    int B;

    // Density of the level-l cell (i, j, k): zero outside the box; a
    // position without a level-l cell reads the covering coarser leaf.
    __device__ __forceinline__ float density(int l, int64_t i, int64_t j, int64_t k) const {
        int64_t n = (int64_t)1 << l;
        if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n) return 0.f;
        while (l > B) {
            const int64_t pi = i >> 1, pj = j >> 1, pk = k >> 1;
            const int64_t np = n >> 1;
            const int32_t o = octidx[l][(pk * np + pj) * np + pi];
            if (o >= 0) return den[l][(int64_t)o * 8 + ((i & 1) | ((j & 1) << 1) | ((k & 1) << 2))];
            i = pi;
            j = pj;
            k = pk;
            n = np;
            --l;
        }
        const int64_t S = n + 2 * kHalo;
        return lev[l][((k + kHalo) * S + (j + kHalo)) * S + (i + kHalo)];
    }
};

// Arguments of the generic per-target-oct FP32 kernel: for each target oct
// (level of its children, oct coordinates), the child densities through
// tg_src (>= 0: index into octden, < 0: -(1 + index into base)), the output
// row of each child through tg_leaf (-1: not a target), shells dl = 1..3
// from the weight lists (or E), dl >= 4 from the automaton and Q tables.
struct AmrSweepArgs {
    AmrLookupView lk;
    const int32_t* tg_info;
    const int64_t* tg_src;
    const int64_t* tg_leaf;
    int64_t n_tg;
    const float* octden;
    const float* base;  // padded level B
    const int32_t* off[5];  // weight lists with the direction fastest ([combo][len][D])
    const float* w[5];
    int len[5];
    const float* kloc;
    const float* gloc;     // [D][8] internal + local chord by crossed-axis set (mirrored rays)
    const int32_t* sgn;    // [D] sign bits of u
    const float* q[CD_MAX_LEVEL + 1];  // coarse tables of levels 2 .. qtop, 216 codes
    int qtop;
    int qcompact;  // Q_qtop holds only the 64 codes of dl = 4 (qtop == Lmax - 4)
    int8_t next[6][2];
    int8_t dl4[4];
    double box;
    int D;
    const float* E;        // shells dl = 1..3 computed by a tiled or split kernel, or nullptr
    const int64_t* erow;   // row of E per target (-1: lists), or nullptr: row g
    int all_rows;          // every target has a row of E (no -1 in erow)
    const float* x4;       // in-situ mode: shells dl >= 4 per target [n_tg][D] (instead of the q tables)
    float* N;
    float* chi;
    float chi_scale;
};

void launch_target_octs(const AmrSweepArgs& a, hipStream_t s);

void launch_amr_external_mfma(const AmrLookupView& lk, const int32_t* tg_info, const int32_t* grp,
                              const int32_t* grp_info, int64_t ngroups, const cd_weights* w, double box, float* E,
                              hipStream_t s);

int amr_layout(cd_tree* t, const int64_t* n_octs, const int32_t* const* oct_parents, int64_t n_leaf,
               hipStream_t s);
int amr_update(cd_tree* t, const float* leaf_n_dev, hipStream_t s);
int amr_leaf_coords(const cd_tree* t, int8_t* level, int32_t* ijk);
int amr_columns(cd_tree* t, const cd_weights* w, float* N, float* chi, float chi_scale, hipStream_t s);
void amr_free(cd_tree* t);
int build_dense_below(cd_tree* t, int top, hipStream_t s);
int alloc_dense_levels(cd_tree* t, int top, hipStream_t s);
int alloc_sweep_buffers(cd_tree* t, int top, int64_t ext_rows, int64_t insitu_rows, float** insitu);
int tree_layout(cd_tree* t, const int64_t* n_octs, const int32_t* const* oct_parents, int64_t n_leaf,
                hipStream_t s);
int count_invalid(const float* v, int64_t n, unsigned long long* counter, int64_t* out, hipStream_t s);
int build_uniform_pyramid(cd_tree* t, hipStream_t s);
}  // namespace cd
