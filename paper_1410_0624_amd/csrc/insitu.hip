// In-situ reference points (Sect. 4.4): every shell is seen from the centre
// of the target's oct, with no tabulated geometry.  The shells dl = 1, 2, 3
// already use that point in the precalculated scheme (the 73 configurations
// of Sect. 3.3 differ from it only for dl >= 4), so the tiled kernels keep
// computing them; this pass adds, per oct and direction, the shells of
// levels L-4 .. 0, each the box between two consecutive outer limits
// (Sect. 3.2), by walking the ray from the oct centre through the shell's
// cells: sum of n x (length of the ray inside the cell), in FP64.
#include <cmath>

#include "cd_internal.h"

namespace cd {

struct InsituArgs {
    const float* lev[CD_MAX_LEVEL + 1];  // padded levels 0 .. L-4
    int L;                                // leaf level; octs at L-1
    const double* dirs;                   // [D][6]: u, then 1 / u per axis (0 where u has no component)
    int D;
    double box;                           // cm
    float* E;                             // [n_oct][D]
    int accumulate;                       // 1: added to E, 0: written
    int64_t n_oct;
};

// The oct A's (level l0 - 1 coordinates, targets at level l0) centre c in
// box units and the inner limit of its level-(l0 - 4) shell: the outer
// limits of the shells dl = 1, 2, 3 (the same for every direction).
struct InsituOct {
    double c[3];
    int64_t ilo[3], ihi[3];
};

__device__ __forceinline__ InsituOct insitu_oct(int l0, const int64_t (&A)[3]) {
    InsituOct o;
    const int L1 = l0 - 1;
    for (int k = 0; k < 3; ++k) {
        int64_t lo = A[k], hi = A[k];
        for (int l = L1; l > L1 - 3; --l) {
            int64_t olo = lo - 2, ohi = hi + 2;
            if (olo & 1) olo -= 1;  // the outer box covers whole parent cells
            if (!(ohi & 1)) ohi += 1;
            lo = olo / 2;           // olo is even, ohi + 1 is even
            hi = (ohi + 1) / 2 - 1;
        }
        o.ilo[k] = lo;
        o.ihi[k] = hi;
        o.c[k] = ((double)A[k] + 0.5) * ldexp(1.0, -L1);
    }
    return o;
}

// Column (box units x density) of the in-situ shells dl >= 4 of the oct
// along u: the levels l0 - 4 .. 0 of the padded arrays lev.  Each shell is
// walked cell by cell from the ray's exit of the inner box to its exit of
// the outer box, the next crossing per axis advanced by one cell's extent
// along the ray.  The inner box of a shell is the outer box of the shell
// below (both limits are whole cells of the coarser level), so its exit is
// the previous shell's outer exit, bit for bit.  Cell indexes fit 32 bits:
// the walked levels are at most CD_MAX_LEVEL - 4.
__device__ double insitu_column(const float* const* lev, int l0, const InsituOct& oc, const double (&u)[3],
                                const double (&iu)[3]) {
    const int L1 = l0 - 1;
    if (L1 - 3 < 0) return 0.0;
    int ilo[3] = {(int)oc.ilo[0], (int)oc.ilo[1], (int)oc.ilo[2]};
    int ihi[3] = {(int)oc.ihi[0], (int)oc.ihi[1], (int)oc.ihi[2]};
    const double(&c)[3] = oc.c;
    const int sgn[3] = {u[0] > 0.0 ? 1 : (u[0] < 0.0 ? -1 : 0), u[1] > 0.0 ? 1 : (u[1] < 0.0 ? -1 : 0),
                        u[2] > 0.0 ? 1 : (u[2] < 0.0 ? -1 : 0)};
    double sum = 0.0;
    double t_in = -1.0;  // set for the first shell, then the previous shell's outer exit
    for (int l = L1 - 3; l >= 0; --l) {
        const int nl = 1 << l;
        // an inner box that covers the whole level leaves this shell and
        // every coarser one outside the box (no matter there)
        if (ilo[0] <= 0 && ilo[1] <= 0 && ilo[2] <= 0 && ihi[0] >= nl - 1 && ihi[1] >= nl - 1 && ihi[2] >= nl - 1)
            break;
        const double dx = ldexp(1.0, -l), idx_scale = ldexp(1.0, l);
        // per axis only the faces ahead of the ray matter: the inner box's
        // (where the ray leaves it) and the outer box's
        int olo[3], ohi[3], lim[3];
        double t_out = 1e300, fin[3];
        for (int k = 0; k < 3; ++k) {
            olo[k] = ilo[k] - 2;
            ohi[k] = ihi[k] + 2;
            if (olo[k] & 1) olo[k] -= 1;
            if (!(ohi[k] & 1)) ohi[k] += 1;
            lim[k] = sgn[k] > 0 ? ohi[k] + 1 : olo[k] - 1;  // the first index past the outer box ahead
            fin[k] = 1e300;
            if (sgn[k] != 0) {
                fin[k] = ((double)(sgn[k] > 0 ? ihi[k] + 1 : ilo[k]) * dx - c[k]) * iu[k];
                t_out = fmin(t_out, ((double)(sgn[k] > 0 ? ohi[k] + 1 : olo[k]) * dx - c[k]) * iu[k]);
            }
        }
        if (t_in < 0.0) t_in = fmin(fmin(fin[0], fin[1]), fin[2]);
        // first cell past the inner box: the axes that leave it at t_in
        // step out of it by index, the others contain c + t_in u; then the
        // first crossing along each axis and the distance between crossings
        int i[3];
        double tn[3], dt[3];
        for (int k = 0; k < 3; ++k) {
            const double pk = (c[k] + t_in * u[k]) * idx_scale;  // exact: a power of two
            if (fin[k] == t_in) i[k] = sgn[k] > 0 ? ihi[k] + 1 : ilo[k] - 1;
            else i[k] = (int)(sgn[k] < 0 ? ceil(pk) - 1.0 : floor(pk));  // a face hit: the cell ahead
            tn[k] = sgn[k] > 0 ? ((double)(i[k] + 1) * dx - c[k]) * iu[k]
                               : (sgn[k] < 0 ? ((double)i[k] * dx - c[k]) * iu[k] : 1e300);
            dt[k] = sgn[k] != 0 ? dx * fabs(iu[k]) : 0.0;
        }
        const int S = nl + 2 * kHalo;
        const int step[3] = {sgn[0], sgn[1] * S, sgn[2] * S * S};
        const float* lv = lev[l];
        int idx = ((i[2] + kHalo) * S + (i[1] + kHalo)) * S + (i[0] + kHalo);
        double t = t_in;
        // at most (width of the outer box) crossings per axis; the walk
        // stops when a crossing leaves the outer box (the advanced crossing
        // times can round a face crossing to just before t_out)
        for (int n = 0; n < 96 && t < t_out; ++n) {
            const double te = fmin(fmin(fmin(tn[0], tn[1]), tn[2]), t_out);
            sum += (double)lv[idx] * (te - t);
            bool out = false;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (tn[k] == te) {
                    idx += step[k];
                    i[k] += sgn[k];
                    tn[k] += dt[k];
                    out |= i[k] == lim[k];
                }
            if (out) break;
            t = te;
        }
        t_in = t_out;
        for (int k = 0; k < 3; ++k) {
            ilo[k] = olo[k] / 2;
            ihi[k] = (ohi[k] + 1) / 2 - 1;
        }
    }
    return sum;
}

__global__ __launch_bounds__(256) void k_insitu_coarse(const InsituArgs a) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= a.n_oct) return;
    const int L1 = a.L - 1;
    const int64_t n1 = (int64_t)1 << L1;
    const int64_t A[3] = {o & (n1 - 1), (o >> L1) & (n1 - 1), o >> (2 * L1)};
    float* row = a.E + o * a.D;
    const InsituOct oc = insitu_oct(a.L, A);
    for (int d = 0; d < a.D; ++d) {
        const double u[3] = {a.dirs[6 * d], a.dirs[6 * d + 1], a.dirs[6 * d + 2]};
        const double iu[3] = {a.dirs[6 * d + 3], a.dirs[6 * d + 4], a.dirs[6 * d + 5]};
        const float v = (float)(insitu_column(a.lev, a.L, oc, u, iu) * a.box);
        row[d] = a.accumulate ? row[d] + v : v;
    }
}

// Adaptive trees: the in-situ shells dl >= 4 of every target oct (level of
// its targets and oct coordinates in info[4 g .. 4 g + 3]) into X[g][D]; a
// thread per target oct and chunk of up to kInsituChunk directions
// (blockIdx.y), so that a tree with few target octs still fills the GPU.
// On uniform grids a thread keeps the whole row: the octs alone fill the
// GPU there, and rows split over threads measured slower.
constexpr int kInsituChunk = 4;

__global__ __launch_bounds__(256) void k_insitu_targets(const InsituArgs a, const int32_t* __restrict__ info,
                                                        int64_t n_tg, float* __restrict__ X) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_tg) return;
    const int l0 = info[4 * g];
    const int64_t A[3] = {info[4 * g + 1], info[4 * g + 2], info[4 * g + 3]};
    const InsituOct oc = insitu_oct(l0, A);
    const int d0 = (int)blockIdx.y * kInsituChunk, d1 = min(a.D, d0 + kInsituChunk);
    for (int d = d0; d < d1; ++d) {
        const double u[3] = {a.dirs[6 * d], a.dirs[6 * d + 1], a.dirs[6 * d + 2]};
        const double iu[3] = {a.dirs[6 * d + 3], a.dirs[6 * d + 4], a.dirs[6 * d + 5]};
        X[g * a.D + d] = (float)(insitu_column(a.lev, l0, oc, u, iu) * a.box);
    }
}

// The in-situ shells dl >= 4 of every oct of a uniform 2^L grid (L >= 4),
// added to E or written into it.
void launch_insitu_coarse(const cd_tree* t, const cd_weights* w, float* E, bool accumulate, hipStream_t s) {
    const int L = t->lmax;
    if (L - 4 < 0) return;
    InsituArgs a{};
    for (int l = 0; l <= L - 4; ++l) a.lev[l] = t->lev[l];
    a.L = L;
    a.dirs = w->dirs;
    a.D = w->D;
    a.box = t->box_cm;
    a.E = E;
    a.accumulate = accumulate ? 1 : 0;
    a.n_oct = (int64_t)1 << (3 * (L - 1));
    k_insitu_coarse<<<(unsigned)((a.n_oct + 255) / 256), 256, 0, s>>>(a);
}

void launch_insitu_targets(const cd_tree* t, const cd_weights* w, const int32_t* info, int64_t n_tg, float* X,
                           hipStream_t s) {
    if (n_tg <= 0) return;
    InsituArgs a{};
    for (int l = 0; l <= t->lmax - 1; ++l) a.lev[l] = t->lev[l];  // every level below Lmax is dense
    a.L = t->lmax;
    a.dirs = w->dirs;
    a.D = w->D;
    a.box = t->box_cm;
    const dim3 grid((unsigned)((n_tg + 255) / 256), (unsigned)((a.D + kInsituChunk - 1) / kInsituChunk));
    k_insitu_targets<<<grid, 256, 0, s>>>(a, info, n_tg, X);
}

}  // namespace cd
