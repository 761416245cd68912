/*
 * colden: tree-based column densities on a fully threaded octree, for AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Valdivia & Hennebelle (2014), "A fast tree-based method for
 * estimating column densities in Adaptive Mesh Refinement codes", A&A.
 * For every leaf (target) cell and every direction sector the column
 *   N(m,n) = sum_i n_i dx_i(m,n)                                 (Eq. 8)
 * is split into the internal + local part (the target and its 7 siblings,
 * rays from the target centre) and the external part, a sum over concentric
 * cubic shells, one per coarser level, whose cells are weighted by
 * precalculated geometric factors K (Sect. 3.2 and 3.3, Eqs. 9-11):
 *   N_ext(m,n) = sum_l dx_l sum_{i in C_l} n_i K(r_i - r_target, m, n, dl).
 * The attenuation factor is chi = (1/D) sum_d exp(-gamma A_V,d) with
 * A_V = N av_per_nh (Eq. 7; gamma = 3.74 and av_per_nh = 1/1.87e21 cm^2
 * reproduce the paper's sigma = 2e-21 cm^2).
 *
 * Conventions for every call:
 *  - Status codes: CD_OK (0) or a negative CD_E* value; cd_last_error()
 *    returns a thread-local message for the last failure.  Nothing aborts,
 *    nothing throws across this boundary.
 *  - Pointers named *_dev are device pointers (HIP global memory); every
 *    other pointer is host memory.  The caller owns every buffer it passes.
 *    Device memory of the tree and weight handles is a workspace the caller
 *    allocates (its size from cd_tree_workspace_bytes and
 *    cd_weights_workspace_bytes) and keeps alive until the handle is
 *    destroyed; the library owns only the host side of a handle.  Nothing on
 *    the cd_tree_update / cd_column_densities / cd_screening_factor /
 *    cd_check_densities path allocates device memory or creates a stream.
 *    (The surrogate handle, not part of the paper's method, owns its own.)
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    asynchronous on that stream; host arguments are consumed before return.
 *    A second stream for stages that run side by side may be given to a
 *    tree (cd_tree_set_aux_stream); the library creates none.
 *  - Leaf order (input densities, output rows): base-level cells in row-major
 *    order (x fastest) skipping refined ones, then for each finer level the
 *    octs in the order given, each oct's children c = i + 2j + 4k (i, j, k
 *    the x, y, z child bits) skipping refined ones.  A uniform 2^L grid
 *    (base_level == max_level) is plain row-major order.
 *  - Densities are in cm^-3, columns in cm^-2; densities must be finite and
 *    >= 0: cd_build_tree checks them (CD_EINVAL), cd_tree_update does not
 *    (cd_check_densities counts the offending entries of any buffer).
 *  - Boundary: non-periodic; no matter outside the box.
 */
#ifndef COLDEN_H
#define COLDEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CD_OK = 0,
    CD_EINVAL = -1,       /* invalid argument */
    CD_ENOMEM = -2,       /* device or host allocation failed */
    CD_EDEVICE = -3,      /* HIP runtime or kernel launch error */
    CD_EUNSUPPORTED = -4  /* valid but not provided by this build */
};

/* direction families */
enum {
    CD_DIR_HEALPIX = 0,   /* HEALPix ring-scheme pixel centres, p1 = Nside: 12 Nside^2 sectors */
    CD_DIR_PAPER_MN = 1,  /* the paper's M x N grid (Sect. 3.2, Eqs. 5-6), p1 = M, p2 = N */
    CD_DIR_AXES6 = 2      /* +x, -x, +y, -y, +z, -z (Sect. 4.4) */
};

/* reference-point modes */
enum {
    CD_PRECALC73 = 0,     /* two-level approximation, 73 configurations (Sect. 3.3) */
    CD_INSITU = 1         /* reference at the oct centre for every shell (Sect. 4.4) */
};

/* contraction precision */
enum {
    CD_FP32 = 0,          /* FP32 densities and weights, FP32 accumulation */
    CD_BF16X2 = 1,        /* densities and weights split hi+lo in bf16, MFMA, FP32 accumulation */
    CD_FP16X2 = 2         /* same with fp16 and a per-tile power-of-two density scale */
};

#define CD_MAX_DIRS 128
#define CD_MAX_LEVEL 12

typedef struct cd_tree cd_tree;
typedef struct cd_weights cd_weights;

/* Thread-local message describing the last failed call ("" if none). */
const char* cd_last_error(void);

/* ABI version (incremented on incompatible changes). */
int cd_version(void);

/*
 * Direction set of a family (Sect. 3.2).  Writes D unit vectors, row d =
 * (ux, uy, uz), into out[capacity][3] and sets *D.  Components with
 * |u_k| < 1e-14 are set to 0.
 * Errors: CD_EINVAL for unknown scheme, p1/p2 < 1, or capacity < D.
 */
int cd_directions(int scheme, int p1, int p2, double* out, int capacity, int* D);

/*
 * Device bytes of the workspace a tree of this structure needs: the dense
 * padded pyramid levels, the index maps and target lists of an adaptive tree,
 * and the sweep's buffers for up to max_dirs directions (per-oct rows of the
 * external shells dl = 1..3, the coarse tables of the shells dl >= 4, the
 * in-situ rows, a check counter).  Host only: touches no device.  Arguments
 * as cd_build_tree.  Errors: CD_EINVAL (malformed structure, NULL bytes).
 */
int cd_tree_workspace_bytes(int base_level, int max_level, const int64_t* n_octs,
                            const int32_t* const* oct_parents, int64_t n_leaf, int max_dirs, size_t* bytes);

/*
 * Build the tree of a fully threaded octree and its pyramid (Sect. 3: a
 * coarse cell holds the mean of its 8 children).
 *   box_cm           edge of the cubic box in cm; dx_l = 0.5^l box_cm.
 *   base_level       B: level of the full base grid (2^B cells per axis).
 *   max_level        Lmax >= B, at most CD_MAX_LEVEL.
 *   n_octs           host [Lmax - B] oct counts of levels B+1 .. Lmax (NULL if Lmax == B).
 *   oct_parents      host [Lmax - B] pointers; level l's array is int32
 *                    [n_octs][3] (x, y, z) of the refined parent cells at
 *                    level l-1; each parent must exist.
 *   leaf_n_dev       device float [n_leaf] leaf densities in leaf order.
 *                    A uniform grid keeps reading this buffer in every
 *                    later cd_column_densities until the next
 *                    cd_tree_update: keep it alive and unchanged (and
 *                    8-byte aligned, else CD_EINVAL).  An AMR tree copies
 *                    the leaves.
 *   n_leaf           number of leaves implied by the structure.
 *   max_dirs         1 .. CD_MAX_DIRS: the largest direction count the tree
 *                    will be swept with (cd_column_densities rejects more).
 *   workspace_dev    device memory of at least cd_tree_workspace_bytes bytes,
 *                    256-byte aligned, owned by the caller, alive and not
 *                    used for anything else until cd_tree_destroy.
 * The structure is copied; the pyramid is built on `stream`.  The leaf
 * densities are checked (finite, >= 0), which synchronises `stream`.
 * Errors: CD_EINVAL (malformed structure, wrong n_leaf, a density that is
 * negative, NaN or infinite, a workspace that is too small or misaligned),
 * CD_EDEVICE.
 */
int cd_build_tree(double box_cm, int base_level, int max_level,
                  const int64_t* n_octs, const int32_t* const* oct_parents,
                  const float* leaf_n_dev, int64_t n_leaf, int max_dirs,
                  void* workspace_dev, size_t workspace_bytes, void* stream, cd_tree** out);

/*
 * Second stream of a tree's sweep: cd_column_densities then runs the coarse
 * tables (and, on adaptive trees, the gathered targets) beside the external
 * shells, and the rows of one z-slab beside the external shells of the next,
 * joining `stream` of the call before it returns.  NULL (the default): every
 * stage runs on the call's stream, one after the other.  The stream must
 * outlive the tree's use; keep it at the default priority.
 * Errors: CD_EINVAL (NULL tree).
 */
int cd_tree_set_aux_stream(cd_tree* tree, void* stream);

/* Number of entries of leaf_n_dev[n_leaf] (device float) that are
 * negative, NaN or infinite, written to *n_invalid; -0.0 and subnormal
 * values are valid.  scratch_dev: 8 bytes of device memory (8-byte aligned)
 * the count is accumulated in.  Synchronises `stream`.
 * Errors: CD_EINVAL (NULL n_invalid or scratch, n_leaf < 0, NULL buffer with
 * n_leaf > 0), CD_EDEVICE. */
int cd_check_densities(const float* leaf_n_dev, int64_t n_leaf, void* scratch_dev, int64_t* n_invalid,
                       void* stream);

/* cd_check_densities for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops): the same count, accumulated
 * in a 256-byte scratch array the library holds per GPU (in device memory
 * from load until the process ends) instead of a caller scratch.  n_leaf is
 * not limited by it (the count is 64-bit).  Calls that overlap on one GPU
 * share that array and race: run them one after another.  Allocates nothing;
 * synchronises `stream`.
 * Errors: CD_EINVAL (NULL n_invalid, n_leaf < 0, NULL buffer with n_leaf >
 * 0), CD_EDEVICE. */
int cd_check_densities_noalloc(const float* leaf_n_dev, int64_t n_leaf, int64_t* n_invalid, void* stream);

/* New leaf densities for an existing structure (one hydro step later):
 * rebuilds the pyramid on `stream`.  n_leaf must be the tree's leaf count.
 * Same layout and lifetime rules as cd_build_tree.
 * Errors: CD_EINVAL (NULL arguments, wrong n_leaf, misaligned buffer). */
int cd_tree_update(cd_tree* tree, const float* leaf_n_dev, int64_t n_leaf, void* stream);

/* Number of leaves of the tree. */
int cd_tree_n_leaf(const cd_tree* tree, int64_t* n_leaf);

/* Level (int8) and (x, y, z) coordinates (int32) of every leaf, host buffers
 * [n_leaf] and [n_leaf][3]. */
int cd_tree_leaf_coords(const cd_tree* tree, int8_t* level, int32_t* ijk);

/* Release the handle (after the stream's work that uses it has completed);
 * its workspace then returns to the caller.  NULL is ignored. */
void cd_tree_destroy(cd_tree* tree);

/*
 * Precalculated geometric weights (Sect. 3.3): for the 73 reference
 * configurations and every cell of the 11^3 standard cube, the distance a
 * ray along each direction crosses in that cell (in cell widths), restricted
 * to the cells of each shell shape, computed once in double precision on the
 * host and uploaded once.  Also the internal + local weights of a target's
 * own oct.
 *   dirs       host [D][3] unit vectors (|u| = 1 within 1e-9).
 *   D          1 .. CD_MAX_DIRS.
 *   mode       CD_PRECALC73: shells dl >= 3 seen from the 73 reference
 *              configurations of Sect. 3.3 (tabulated, coarse tables for
 *              dl >= 4); CD_INSITU: every shell seen from the centre of
 *              the target's oct (Sect. 4.4).  The two differ only for
 *              dl >= 4, which the in-situ form computes per target oct by
 *              walking each ray through the shells' cells (FP64), on
 *              uniform grids and adaptive trees, for any D; with a split
 *              precision it has the split forms' own limits (below).
 *   precision  CD_FP32, CD_BF16X2 or CD_FP16X2: the arithmetic of the
 *              external shells dl = 1, 2, 3 in cd_column_densities.  The
 *              split forms keep densities and weights as hi + lo pairs of
 *              16-bit halves (rounded from the FP64 weights here) and run
 *              the contraction on the matrix cores with FP32 accumulation;
 *              measured error |d ln N| <= 3e-5 (bf16) and <= 1e-6 (fp16).
 *              CD_FP16X2 divides each LDS density tile by a power of two:
 *              it needs the tiled kernel, i.e. D in {6, 12, 24, 40, 48}, and
 *              on uniform grids 2^L >= 32.  CD_BF16X2 on uniform grids
 *              needs the same; on adaptive trees it takes any D.  On
 *              adaptive trees the split forms cover the targets of the
 *              16^3-oct tiles that the tiled kernel sweeps (the densely
 *              occupied ones); the other targets (sparse tiles, levels
 *              without tiles) are gathered in FP32 in every form, except
 *              that CD_BF16X2 for a D outside that set gathers every target
 *              on the matrix cores.
 *   workspace_dev  device memory of at least cd_weights_workspace_bytes
 *              bytes for the same arguments, 256-byte aligned, owned by the
 *              caller and kept until cd_weights_destroy.
 * The tables are copied into the workspace on `stream`, which is then
 * synchronised.
 * Errors: CD_EINVAL (bad arguments, a workspace that is too small or
 * misaligned), CD_EUNSUPPORTED, CD_EDEVICE.
 */
int cd_precompute_weights(const double* dirs, int D, int mode, int precision,
                          void* workspace_dev, size_t workspace_bytes, void* stream, cd_weights** out);

/* Device bytes of the workspace cd_precompute_weights needs for these
 * arguments (host only: the tables are computed, nothing is uploaded).
 * Errors: as cd_precompute_weights. */
int cd_weights_workspace_bytes(const double* dirs, int D, int mode, int precision, size_t* bytes);

/*
 * The precalculated geometric factors K of Sect. 3.3 (Eqs. 10-11) as the
 * library computes them in FP64 on the host before cd_precompute_weights
 * rounds and uploads them; a host-only query that touches no device.
 *   kind 1, 2, 3: the shells dl = 1, 2, 3; kind 4: dl >= 4; kind 0: the
 *   internal + local factors of the target's own oct (Sect. 3.2).
 * Shells (kind 1..4): combo c indexes the per-axis shapes x + na (y + na z)
 * (na = 2, 4, 8, 12 shapes per axis: parity of the level-l ancestor A_l,
 * octant bits of A_(l+1), A_(l+2), and for kind 4 the inner-limit state).
 * For each (c, d) the cnt[c][d] non-zero entries: off[c][d][e][3] the cell
 * offset from A_l (level-l cells, each in -5..5: the 11^3 standard cube),
 * w[c][d][e] the chord of the ray from the reference point along u_d through
 * that cell, in level-l cell widths; entries e >= cnt are zero padding.
 * ref[c][3] is the reference point relative to the centre of A_l and
 * box[c][3][4] = (inner lo, inner hi, outer lo, outer hi) per axis: the
 * entries are the cells of the outer box that are not in the inner box.
 * Kind 0: c = octant a of the target (bits x, y, z), entries e = the 8 cells
 * of the oct (off = their bits), w = chord from the target centre ref[a]
 * (oct coordinates, cell width 1) through each cell; box unused.
 * Call with off == NULL to get *ncombo and *len (entries per (c, d)); then
 * off [ncombo][D][len][3], w [ncombo][D][len], cnt [ncombo][D], ref
 * [ncombo][3], box [ncombo][3][4] (host buffers; w, cnt, ref, box may be NULL).
 * Errors: CD_EINVAL (NULL dirs/ncombo/len, D or kind out of range, a
 * direction that is not a unit vector),
 * CD_EUNSUPPORTED (a direction set needing more than 12 entries per coarse list).
 */
int cd_weight_lists(const double* dirs, int D, int kind, int* ncombo, int* len, int32_t* off, double* w,
                    int32_t* cnt, double* ref, int32_t* box);

/* Number of directions of a weights handle. */
int cd_weights_n_dirs(const cd_weights* w, int* D);

/*
 * Size of the split-precision contraction (cost model): the number of steps
 * of 32 shell offsets summed over the 64 configuration classes (A mod 4 per
 * axis), the shells dl = 1, 2, 3 and the tiles of 16 directions.  On a
 * uniform grid a tile of 16^3 octs runs steps x 4 row blocks x 3 matrix
 * instructions of 16 x 16 x 32 (bf16 or fp16) for those shells.  0 for
 * CD_FP32 weights.
 * Errors: CD_EINVAL (NULL argument).
 */
int cd_weights_split_steps(const cd_weights* w, int64_t* steps);

/* Release the handle (after the stream's work that uses it); its workspace
 * then returns to the caller. */
void cd_weights_destroy(cd_weights* w);

/*
 * Column densities of every leaf (Eqs. 8-11): writes N_dev[n_leaf][D]
 * (float, cm^-2, row-major, direction fastest).  If chi_dev is not NULL the
 * screening factor (Eq. 7) is fused and written to chi_dev[n_leaf]
 * using av_per_nh and gamma (ignored otherwise).  The contraction runs in
 * the precision of the weights handle (see cd_precompute_weights); the
 * coarse shells (dl >= 4), the internal + local part, the level sums and chi
 * are FP32 in every form.  N_dev must be 16-byte aligned and chi_dev 8-byte
 * aligned (any device allocation is).  Asynchronous on `stream`.
 * Allocates nothing: its intermediates live in the tree's workspace.
 * Errors: CD_EINVAL (NULL handles or output, misaligned buffers, more
 * directions than the tree's max_dirs), CD_EUNSUPPORTED (a split form on a
 * tree it is not offered for), CD_EDEVICE.
 */
int cd_column_densities(cd_tree* tree, const cd_weights* w, float* N_dev, float* chi_dev,
                        double av_per_nh, double gamma, void* stream);

/*
 * The same sweep with the columns written in a packed 16-bit format, half
 * the bytes of N (an output format, not part of the paper's method; the
 * sums and chi are those of cd_column_densities, chi from the FP32 columns):
 * Ncode_dev[n_leaf][D] (uint16, row-major, direction fastest) holds
 *   c = round(1024 (log2 N - 40)), clamped to 0 .. 65535,
 * so N = 2^(40 + c / 1024) to within 2^-11 in log2 (|d ln N| <= 3.4e-4)
 * for 2^40 (1.1e12 cm^-2) <= N <= 2^104; smaller columns give c = 0.
 * Uniform grids of 2^L >= 32 cells per axis, D in {12, 24, 40, 48}, any
 * precision and mode of the weights.  Ncode_dev 16-byte and chi_dev 8-byte
 * aligned.  Asynchronous on `stream`; allocates nothing.
 * Errors: CD_EINVAL (NULL handles or output, misaligned buffers),
 * CD_EUNSUPPORTED (adaptive tree, other D or a smaller grid), CD_EDEVICE.
 */
int cd_column_densities_log16(cd_tree* tree, const cd_weights* w, uint16_t* Ncode_dev, float* chi_dev,
                              double av_per_nh, double gamma, void* stream);

/*
 * Screening factor (Eq. 7): A_V = N av_per_nh, chi = (1/D) sum_d
 * exp(-gamma A_V,d).  N_dev [n_leaf][D]; writes chi_dev[n_leaf] and, if not
 * NULL, av_dev[n_leaf][D].  Asynchronous on `stream`.
 * Errors: CD_EINVAL (n_leaf < 0, D outside 1..CD_MAX_DIRS, NULL buffers).
 */
int cd_screening_factor(const float* N_dev, int64_t n_leaf, int D, double av_per_nh,
                        double gamma, float* chi_dev, float* av_dev, void* stream);

/*
 * Gas heating from the screening factor (Sect. 5), per cell:
 *   G0_eff = chi G0 (G0 = 1.7 for the Draine field in Habing units);
 *   Gamma_UV = 1e-24 eps G0_eff n  erg cm^-3 s^-1, photoelectric heating with
 *   the efficiency of Wolfire et al. (1995), x = G0_eff T^(1/2) / n_e:
 *   eps = 4.9e-2 / (1 + (x/1925)^0.73) + 3.7e-2 (T/1e4)^0.7 / (1 + x/5000);
 *   Gamma_CR = 1e-27 n  erg cm^-3 s^-1 (cosmic rays).
 * Device float arrays [n_cells]: chi_dev (cd_heating_rates: input), n_dev
 * (cm^-3), T_dev (K), ne_dev (electron density, cm^-3; the paper takes it
 * from a model it does not state, so it is an input here); outputs
 * g0eff_dev and gamma_cr_dev may be NULL.  n_e <= 0 with UV gives eps = 0.
 * Asynchronous on `stream`.
 * Errors: CD_EINVAL (n_cells < 0, NULL buffers, G0 negative or non-finite).
 */
int cd_heating_rates(const float* chi_dev, const float* n_dev, const float* T_dev, const float* ne_dev,
                     int64_t n_cells, double G0, float* g0eff_dev, float* gamma_uv_dev, float* gamma_cr_dev,
                     void* stream);

/*
 * Screening factor (Eq. 7) fused with the heating rates: reads each cell's
 * row of N_dev [n_cells][D] once, writes chi_dev (may be NULL) and the rates
 * as cd_heating_rates.  Errors: CD_EINVAL (as cd_heating_rates, D outside
 * 1..CD_MAX_DIRS, non-finite av_per_nh or gamma).
 */
int cd_screening_heating(const float* N_dev, int64_t n_cells, int D, double av_per_nh, double gamma,
                         const float* n_dev, const float* T_dev, const float* ne_dev, double G0, float* chi_dev,
                         float* g0eff_dev, float* gamma_uv_dev, float* gamma_cr_dev, void* stream);

/*
 * Stage timing.  When enabled on a tree, cd_column_densities and
 * cd_tree_update record HIP events around each of their stages on the
 * streams the stages run on; cd_profile_read waits for the last call's events
 * and returns the stage durations in milliseconds (0 for a stage that did not
 * run).  Stages: CD_STAGE_PYRAMID (cd_tree_update), CD_STAGE_COARSE (shells
 * dl >= 4), CD_STAGE_EXTERNAL (shells dl = 1..3), CD_STAGE_ROWS (internal +
 * local, N and chi), CD_STAGE_SWEEP (the whole cd_column_densities call).
 * When a uniform sweep runs in z-slabs (its two kernels overlapping), the
 * external and row stages are the sums of their launches.
 * Errors: CD_EINVAL (NULL tree or output), CD_EDEVICE.
 */
enum { CD_STAGE_PYRAMID = 0, CD_STAGE_COARSE = 1, CD_STAGE_EXTERNAL = 2, CD_STAGE_ROWS = 3, CD_STAGE_SWEEP = 4,
       CD_NUM_STAGES = 5 };
int cd_profile_enable(cd_tree* tree, int on);
int cd_profile_read(cd_tree* tree, float* ms /* [CD_NUM_STAGES] */);


/*
 * Learned surrogate of the column sweep.  Not part of the paper's method: a
 * network trained on the columns the method computes, with the method as
 * fallback.  Uniform grids; a network serves one leaf level L, 8 or 9
 * (2^L = 256 or 512 cells per axis).
 *
 * Features of a leaf (576): for each absolute level l = 0 .. 8 of the
 * pyramid (Sect. 3: a coarse cell holds the mean of its children), the 4^3
 * level-l cells centred on the centre of the leaf's level-(l-1) ancestor A
 * (indices 2A-1 .. 2A+2 per axis; A = 0 at l = 0), feature
 * l*64 + sx + 4 sy + 16 sz = (ln max(n, 1e-10) - in_shift) / in_scale, with
 * n = 0 outside the box.  They depend on the leaf's level-7 ancestor only,
 * so the network runs once per level-7 cell (a "row").  It predicts the
 * near shells dl = 1..3 of the external sum (Sect. 3.2, Eqs. 9-10; shared by
 * the 8 leaves of an oct) of each of the 8^(L-8) octs inside that cell:
 * Dout = 8^(L-8) D outputs, block j = jx + 2^(L-8) (jy + 2^(L-8) jz) of D
 * values for the oct at offset (jx, jy, jz) inside the cell,
 * y = (ln(E + 1e17) - out_shift) / out_scale per direction, E the method's
 * near-shell column.  The method supplies the rest exactly: the internal +
 * local part and the shells dl >= 4 (its coarse tables, Eq. 11), so
 * N = N_il + N_dl>=4 + max(exp(y out_scale + out_shift) - 1e17, 0).
 * The near shells are what the method spends its gather on, and they carry
 * less of the column than the coarse shells, which the 4^3 stencils resolve
 * worst.  Network: 576 -> width -> width -> Dout, ReLU.
 * Loss: mean squared error over all outputs.  Optimiser: Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8).
 * Parameters in the order W1 [576][width], b1, W2 [width][width], b2,
 * W3 [width][Dout], b3 (row-major, y = x W + b), FP32 master copies.
 *
 * CD_SURR_BF16: inference (cd_surrogate_infer, cd_surrogate_forward) with
 * weights and activations rounded to bfloat16 on the matrix cores, FP32
 * accumulation; training (train steps, cd_surrogate_gradients) on the
 * matrix cores too, with every FP32 operand split into bfloat16 hi + lo
 * and three products per pair (about 16 significant bits), so gradients
 * match FP32 arithmetic.  CD_SURR_FP32: every product in FP32 on the vector
 * units (a checking path).  A handle holds scratch for its largest batch;
 * calls on one handle must not overlap.
 */
enum { CD_SURR_FP32 = 0, CD_SURR_BF16 = 1 };
typedef struct cd_surrogate cd_surrogate;

/* New network for D directions on grids of leaf level leaf_level (8 or 9),
 * hidden width (multiple of 16, 16 .. 1024), precision CD_SURR_*,
 * He-uniform weights from `seed`, zero biases.
 * norm = {in_shift, in_scale, out_shift, out_scale} (scales > 0).
 * Errors: CD_EINVAL, CD_ENOMEM. */
int cd_surrogate_create(int D, int leaf_level, int width, int precision, uint64_t seed, const float* norm,
                        cd_surrogate** out);

/* info[5] = {D, leaf level, width, precision, Dout}. */
int cd_surrogate_info(const cd_surrogate* s, int32_t* info);

/* Release the handle (after the stream's work that uses it).  NULL is ignored. */
void cd_surrogate_destroy(cd_surrogate* s);

/* Number of parameters; copies of the FP32 parameters to / from host memory
 * (set_params also clears the Adam moments and step count). */
int cd_surrogate_n_params(const cd_surrogate* s, int64_t* n);
int cd_surrogate_get_params(const cd_surrogate* s, float* params);
int cd_surrogate_set_params(cd_surrogate* s, const float* params);

/* Scaled features of n leaves (row-major leaf indices cells_dev[n], device
 * int64) into X_dev[n][576] (device float).  An index outside [0, n_leaf)
 * gives NaN features (here and in cd_surrogate_train_step).
 * Errors: CD_EINVAL (tree not uniform or 2^L < 256, NULL buffers). */
int cd_surrogate_features(const cd_surrogate* s, const cd_tree* tree, const int64_t* cells_dev, int64_t n,
                          float* X_dev, void* stream);

/* Training targets of n leaves (cells_dev[n]) of a tree of the network's
 * leaf level: T_dev[n][Dout], block j = scaled ln(E + 1e17) of oct j of the
 * listed leaf's level-7 cell, E the method's near shells dl = 1..3 computed
 * here with weights w (FP32, precalculated, the network's D, a direction
 * set the tiled near-shell kernel takes: D in {6, 12, 24, 40, 48}).  An
 * index outside [0, n_leaf) gives NaN.
 * Errors: CD_EINVAL, CD_EUNSUPPORTED. */
int cd_surrogate_targets(const cd_surrogate* s, const cd_tree* tree, const cd_weights* w, const int64_t* cells_dev,
                         int64_t n, float* T_dev, void* stream);

/* Unscaled targets of every level-7 cell of a tree of the network's leaf
 * level: T_rows_dev[2^21][Dout] = ln(E + 1e17) (the table
 * cd_surrogate_train_step_rows reads).  Weights as cd_surrogate_targets.
 * Errors: CD_EINVAL, CD_EUNSUPPORTED. */
int cd_surrogate_row_targets(const cd_surrogate* s, const cd_tree* tree, const cd_weights* w, float* T_rows_dev,
                             void* stream);

/* Network outputs Y_dev[n][Dout] (scaled log columns) of inputs X_dev[n][576]. */
int cd_surrogate_forward(cd_surrogate* s, const float* X_dev, int64_t n, float* Y_dev, void* stream);

/* Loss and gradient of the loss for inputs X_dev[n][576] and targets
 * T_dev[n][Dout] (scaled log columns), without an update: grad[n_params] and
 * *loss in host memory (synchronises the stream). */
int cd_surrogate_gradients(cd_surrogate* s, const float* X_dev, const float* T_dev, int64_t n, float* grad,
                           float* loss, void* stream);

/* One Adam step of learning rate lr on a batch of leaves cells_dev[batch] of
 * a uniform tree of the network's leaf level, with targets as
 * cd_surrogate_targets (the near shells are recomputed on every call).  If
 * loss is not NULL the batch loss before the step is written there
 * (synchronises the stream).  Errors: CD_EINVAL, CD_EUNSUPPORTED. */
int cd_surrogate_train_step(cd_surrogate* s, const cd_tree* tree, const cd_weights* w, const int64_t* cells_dev,
                            int64_t batch, float lr, float* loss, void* stream);

/* The same step on level-7 cells rows_dev[batch] (row-major, x fastest; an
 * index outside [0, 2^21) gives NaN): features from `tree`, a uniform tree
 * of any leaf level >= 8 (they read pyramid levels 0 .. 8 only), targets
 * from a table of cd_surrogate_row_targets scaled by the handle's norm.
 * A 2^8 field refined into 2^9 equal leaves has the same levels 0 .. 8, so
 * its 2^8 tree supplies the features of rows labelled on the 2^9 tree.
 * Errors: CD_EINVAL. */
int cd_surrogate_train_step_rows(cd_surrogate* s, const cd_tree* tree, const float* T_rows_dev,
                                 const int64_t* rows_dev, int64_t batch, float lr, float* loss, void* stream);

/* Columns of every leaf of a uniform tree of the network's leaf level: the
 * network's near shells plus the method's internal + local parts and coarse
 * shells dl >= 4 (weights as cd_surrogate_targets): N_dev[n_leaf][D]
 * (cm^-2) and, if chi_dev is not NULL, chi (Eq. 7) with av_per_nh, gamma.
 * N_dev 16-byte and chi_dev 8-byte aligned.
 * Errors: CD_EINVAL, CD_ENOMEM, CD_EUNSUPPORTED. */
int cd_surrogate_infer(cd_surrogate* s, cd_tree* tree, const cd_weights* w, float* N_dev, float* chi_dev,
                       double av_per_nh, double gamma, void* stream);

/* Sampled check and fallback after cd_surrogate_infer: the grid is cut into
 * tiles of 8^3 leaves; in each, ceil(frac * 512) leaves drawn from `seed`
 * are computed with the method (FP32 weights w); a tile where a sample's chi
 * differs from the network's by more than tol_chi (relative) is recomputed
 * entirely with the method (N and chi).  Writes the number of such tiles and
 * of all tiles, and the largest sampled relative chi error (may be NULL).
 * When more than a quarter of the tiles fail, the method runs once over the
 * whole grid straight into N_dev and chi_dev instead, so every tile then holds
 * the method's values.  The tiles are judged on the device; the stream is
 * synchronised once, for the count of failing tiles, and the recomputation
 * is left queued on it.  The sample and tile lists live in the handle
 * (grown on first use).  N_dev 16-byte and chi_dev 8-byte aligned.
 * Errors: CD_EINVAL (frac outside (0, 1], tree not uniform, w not FP32,
 * misaligned buffers), CD_ENOMEM, CD_EDEVICE. */
int cd_surrogate_check_fallback(cd_surrogate* s, cd_tree* tree, const cd_weights* w, double frac, double tol_chi,
                                uint64_t seed, float* N_dev, float* chi_dev, double av_per_nh, double gamma,
                                int64_t* n_fallback_tiles, int64_t* n_tiles, float* max_sample_err, void* stream);

/* Parameters, Adam state and settings to / from a file. */
int cd_surrogate_save(const cd_surrogate* s, const char* path);
int cd_surrogate_load(const char* path, cd_surrogate** out);

#ifdef __cplusplus
}
#endif

#endif /* COLDEN_H */
