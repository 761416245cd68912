// Host geometry of the tree method: direction sets, per-axis shell shapes and
// the precalculated weight tables (Sect. 3.2-3.3), all in double precision.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "cd_internal.h"

namespace cd {

// ------------------------------------------------------------- directions --
static void set_unit(std::array<double, 3>& u, double z, double phi) {
    double s = std::sqrt(std::max(0.0, (1.0 - z) * (1.0 + z)));
    u = {s * std::cos(phi), s * std::sin(phi), z};
    for (double& c : u)
        if (std::fabs(c) < 1e-14) c = 0.0;
}

// HEALPix ring scheme by pixel index (Gorski et al. 2005): north cap rings
// i < Ns hold 4i pixels, the belt rings Ns <= i <= 3Ns hold 4Ns pixels, and
// the south cap mirrors the north one.  Pixels run north to south and by
// increasing azimuth inside a ring.
static void healpix(int ns, std::vector<std::array<double, 3>>& out) {
    const long npix = 12L * ns * ns;
    const long ncap = 2L * ns * (ns - 1);
    out.resize(npix);
    for (long p = 0; p < npix; ++p) {
        double z, phi;
        if (p < ncap) {
            long i = 1;
            while (2 * i * (i + 1) <= p) ++i;  // ring i holds p in [2i(i-1), 2i(i+1))
            long j = p - 2 * i * (i - 1) + 1;
            z = 1.0 - (double)(i * i) / (3.0 * ns * ns);
            phi = M_PI / (2.0 * i) * (j - 0.5);
        } else if (p < npix - ncap) {
            long q = p - ncap;
            long i = q / (4L * ns) + ns;
            long j = q % (4L * ns) + 1;
            int s = (int)((i - ns + 1) & 1);
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * ns);
            phi = M_PI / (2.0 * ns) * (j - 0.5 * s);
        } else {
            long ps = npix - p;  // 1 .. ncap counted from the south pole
            long i = 1;
            while (2 * i * (i + 1) < ps) ++i;
            long j = 2 * i * (i + 1) - ps + 1;
            z = -(1.0 - (double)(i * i) / (3.0 * ns * ns));
            phi = M_PI / (2.0 * i) * (j - 0.5);
        }
        set_unit(out[p], z, phi);
    }
}

int make_directions(int scheme, int p1, int p2, std::vector<std::array<double, 3>>& out) {
    out.clear();
    if (scheme == CD_DIR_HEALPIX) {
        if (p1 < 1 || 12L * p1 * p1 > CD_MAX_DIRS * 64L) return CD_EINVAL;
        healpix(p1, out);
    } else if (scheme == CD_DIR_PAPER_MN) {
        // Sect. 3.2, Eq. 3: theta_m = arccos(1 + (1 - 2m)/M), phi_n = 2 pi (n-1)/N
        if (p1 < 1 || p2 < 1 || (long)p1 * p2 > CD_MAX_DIRS * 64L) return CD_EINVAL;
        for (int m = 1; m <= p1; ++m)
            for (int n = 1; n <= p2; ++n) {
                std::array<double, 3> u;
                set_unit(u, 1.0 + (1.0 - 2.0 * m) / p1, 2.0 * M_PI * (n - 1) / p2);
                out.push_back(u);
            }
    } else if (scheme == CD_DIR_AXES6) {
        out = {{{1, 0, 0}}, {{-1, 0, 0}}, {{0, 1, 0}}, {{0, -1, 0}}, {{0, 0, 1}}, {{0, 0, -1}}};
    } else {
        return CD_EINVAL;
    }
    return CD_OK;
}

// ------------------------------------------------------------------ chord --
double chord(const double lo[3], const double hi[3], const double o[3], const double u[3]) {
    double tin = 0.0, tout = HUGE_VAL;
    for (int k = 0; k < 3; ++k) {
        if (u[k] != 0.0) {
            double inv = 1.0 / u[k];
            double t1 = (lo[k] - o[k]) * inv, t2 = (hi[k] - o[k]) * inv;
            tin = std::max(tin, std::min(t1, t2));
            tout = std::min(tout, std::max(t1, t2));
        } else if (o[k] <= lo[k] || o[k] >= hi[k]) {
            return 0.0;
        }
    }
    return tout > tin ? tout - tin : 0.0;
}

// ----------------------------------------------------------- shell shapes --
// Outer limit of a shell (Sect. 3.2): beyond the inner limit take two or three
// level-l cells so that the outer box covers whole parent (level l-1) cells.
// With p the parity of the ancestor index, an offset o is the start of a
// parent cell when p + o is even.
static AxisShape make_shape(int ilo, int ihi, int p, double ref) {
    AxisShape s;
    s.ilo = ilo;
    s.ihi = ihi;
    s.olo = ilo - (((p + ilo) & 1) ? 3 : 2);
    s.ohi = ihi + (((p + ihi + 1) & 1) ? 3 : 2);
    s.ref = ref;
    return s;
}

// Inner-state codes of kind 4: (inner lo, inner hi, b1, b2)
static const int kState[6][4] = {{-2, 1, 0, 0}, {-1, 2, 1, 1}, {-2, 2, 0, 0},
                                 {-2, 2, 0, 1}, {-2, 2, 1, 0}, {-2, 2, 1, 1}};

// Reference offset of the centre of A_{l+2} (octant bits b1 of A_{l+1} in A_l
// and b2 of A_{l+2} in A_{l+1}) from the centre of A_l, in level-l cells.
static double ref2(int b1, int b2) { return 0.5 * (b1 - 0.5) + 0.25 * (b2 - 0.5); }

int axis_codes(int kind) { return kind == 1 ? 2 : kind == 2 ? 4 : kind == 3 ? 8 : 12; }

std::vector<AxisShape> axis_shapes(int kind) {
    std::vector<AxisShape> v;
    for (int p = 0; p < 2; ++p) {
        if (kind == 1) {
            v.push_back(make_shape(0, 0, p, 0.0));
        } else if (kind == 2) {
            for (int b1 = 0; b1 < 2; ++b1) v.push_back(make_shape(-1, 1, p, 0.5 * (b1 - 0.5)));
        } else if (kind == 3) {
            // the inner limit is the dl = 2 outer box halved: [-2,1] if A_{l+1}
            // is a low child, [-1,2] if a high one
            for (int b1 = 0; b1 < 2; ++b1)
                for (int b2 = 0; b2 < 2; ++b2)
                    v.push_back(b1 ? make_shape(-1, 2, p, ref2(b1, b2)) : make_shape(-2, 1, p, ref2(b1, b2)));
        } else {
            for (int s = 0; s < 6; ++s)
                v.push_back(make_shape(kState[s][0], kState[s][1], p, ref2(kState[s][2], kState[s][3])));
        }
    }
    return v;
}

// The inner limit one level coarser is this shell's outer box halved:
// [-2,1] stays while the ancestors are low children, [-1,2] while they are
// high children, anything else becomes [-2,2] for good.
int next_state_code(int s, int p) {
    int lo = kState[s][0], hi = kState[s][1], b1 = kState[s][2];
    AxisShape o = make_shape(lo, hi, p, 0.0);
    // absolute outer [a+olo, a+ohi] with a = 2a' + p, halved: relative to a'
    int nlo = (p + o.olo) / 2;          // p + olo is even
    int nhi = (p + o.ohi + 1) / 2 - 1;  // p + ohi + 1 is even
    int nb1 = p, nb2 = b1;
    for (int c = 0; c < 6; ++c)
        if (kState[c][0] == nlo && kState[c][1] == nhi && kState[c][2] == nb1 && kState[c][3] == nb2)
            return c;
    return -1;
}

int state_code_dl4(int b1, int b2) {
    // inner limit at dl = 3: [-2,1] if A_{l0-2} is a low child (b2 = 0), else
    // [-1,2]; one level coarser it is that shell's outer box halved, with b1
    // the parity of A_{l0-3}
    const int lo = b2 ? -1 : -2, hi = b2 ? 2 : 1;
    AxisShape o = make_shape(lo, hi, b1, 0.0);
    const int nlo = (b1 + o.olo) / 2, nhi = (b1 + o.ohi + 1) / 2 - 1;
    for (int c = 0; c < 6; ++c)
        if (kState[c][0] == nlo && kState[c][1] == nhi && kState[c][2] == b1 && kState[c][3] == b2)
            return c;
    return -1;
}

// ------------------------------------------------------------------ tables --
int build_tables(const std::vector<std::array<double, 3>>& dirs, HostTables& t) {
    const int D = (int)dirs.size();
    t.D = D;
    for (int kind = 1; kind <= 4; ++kind) {
        std::vector<AxisShape> sh = axis_shapes(kind);
        const int na = (int)sh.size();
        const int nc = na * na * na;
        t.ncombo[kind] = nc;
        std::vector<std::vector<std::pair<int32_t, double>>> lists((size_t)nc * D);
        int maxlen = 1;
        for (int c = 0; c < nc; ++c) {
            const AxisShape& X = sh[c % na];
            const AxisShape& Y = sh[(c / na) % na];
            const AxisShape& Z = sh[c / (na * na)];
            const double r[3] = {X.ref, Y.ref, Z.ref};
            for (int oz = Z.olo; oz <= Z.ohi; ++oz)
                for (int oy = Y.olo; oy <= Y.ohi; ++oy)
                    for (int ox = X.olo; ox <= X.ohi; ++ox) {
                        bool in_inner = ox >= X.ilo && ox <= X.ihi && oy >= Y.ilo && oy <= Y.ihi &&
                                        oz >= Z.ilo && oz <= Z.ihi;
                        if (in_inner) continue;
                        const double lo[3] = {ox - 0.5, oy - 0.5, oz - 0.5};
                        const double hi[3] = {ox + 0.5, oy + 0.5, oz + 0.5};
                        for (int d = 0; d < D; ++d) {
                            double k = chord(lo, hi, r, dirs[d].data());
                            if (k > 1e-12) lists[(size_t)c * D + d].push_back({pack_off(ox, oy, oz), k});
                        }
                    }
            for (int d = 0; d < D; ++d) maxlen = std::max(maxlen, (int)lists[(size_t)c * D + d].size());
        }
        t.len[kind] = maxlen;
        t.off[kind].assign((size_t)nc * D * maxlen, pack_off(0, 0, 0));
        t.w[kind].assign((size_t)nc * D * maxlen, 0.0);
        t.cnt[kind].assign((size_t)nc * D, 0);
        for (size_t q = 0; q < lists.size(); ++q) {
            t.cnt[kind][q] = (int32_t)lists[q].size();
            for (size_t e = 0; e < lists[q].size(); ++e) {
                t.off[kind][q * maxlen + e] = lists[q][e].first;
                t.w[kind][q * maxlen + e] = lists[q][e].second;
            }
        }
    }
    // internal + local: rays from the centre of the target (octant a of the
    // oct) through the 8 cells of the oct, in target-cell widths
    t.kloc.assign((size_t)64 * D, 0.0);
    for (int a = 0; a < 8; ++a) {
        const double o[3] = {(a & 1) + 0.5, ((a >> 1) & 1) + 0.5, ((a >> 2) & 1) + 0.5};
        for (int s = 0; s < 8; ++s) {
            const double lo[3] = {(double)(s & 1), (double)((s >> 1) & 1), (double)((s >> 2) & 1)};
            const double hi[3] = {lo[0] + 1, lo[1] + 1, lo[2] + 1};
            for (int d = 0; d < D; ++d) t.kloc[((size_t)a * 8 + s) * D + d] = chord(lo, hi, o, dirs[d].data());
        }
    }
    return CD_OK;
}

}  // namespace cd
