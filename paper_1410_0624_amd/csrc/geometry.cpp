// Host geometry of the tree method: direction sets, per-axis shell shapes and
// the precalculated weight tables (Sect. 3.2-3.3), all in double precision.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "cd_internal.h"
#include "sweep_layout.h"
#include <cstring>
#include <map>

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
        // Sect. 3.2, Eqs. 5-6: theta_m = arccos(1 + (1 - 2m)/M), phi_n = 2 pi (n-1)/N
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
        if (kind == 4) {
            if (maxlen > 12) {
                set_error("direction set needs %d entries per coarse shell list (at most 12 supported)", maxlen);
                return CD_EUNSUPPORTED;
            }
            maxlen = 12;  // fixed length: the coarse kernel unrolls the list
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

namespace cd {

static int32_t fbits(double w) {
    float f = (float)w;
    int32_t b;
    std::memcpy(&b, &f, 4);
    return b;
}

// Tables of the tiled sweep.  For each configuration class c (A mod 4 per
// axis) and direction, the shell entries as (LDS offset relative to the
// lane's base in its level's tile, weight): dl = 1, dl = 2, and for dl = 3
// the union over the 8 parities of the level L-3 ancestor, split into entries
// common to all parities and entries carrying a parity mask.  Each (class,
// direction) gets one slot of tile::kSlotWords words (layout in
// sweep_layout.h) that the kernel reads with scalar loads.  A list longer than
// its slot part leaves the tiled sweep off for this direction set.
int build_tile_tables(const std::vector<std::array<double, 3>>& dirs, HostTables& t) {
    using namespace tile;
    const int D = (int)dirs.size();
    t.slots.clear();
    t.tile_ok = false;
    // internal + local, for every direction count (the row kernels read
    // these whether or not the tiled sweep takes D): after mirroring u into
    // the positive octant, a target reaches the sibling across axis a only if
    // it lies on the low side of a; the chord through the sibling reached
    // across the axis set m is the same for every target: box [0.5, 1.5]
    // along the crossed axes, [-0.5, 0.5] along the others, ray from the
    // origin along |u|.
    t.gloc.assign((size_t)D * 8, 0.0);
    t.sgn.assign(D, 0);
    for (int d = 0; d < D; ++d) {
        const double au[3] = {std::fabs(dirs[d][0]), std::fabs(dirs[d][1]), std::fabs(dirs[d][2])};
        t.sgn[d] = (dirs[d][0] < 0) | ((dirs[d][1] < 0) << 1) | ((dirs[d][2] < 0) << 2);
        const double org[3] = {0, 0, 0};
        for (int m = 0; m < 8; ++m) {
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = ((m >> a) & 1) ? 0.5 : -0.5;
                hi[a] = lo[a] + 1.0;
            }
            t.gloc[(size_t)d * 8 + m] = chord(lo, hi, org, au);
        }
    }
    std::vector<uint32_t> slots((size_t)64 * D * kSlotWords, 0u);
    // lanes l = lx + 4 ly + 16 lz of each parity p of A >> 2
    uint64_t lanes_of[8] = {0};
    for (int l = 0; l < 64; ++l) {
        const int p = (l & 1) | (((l >> 2) & 1) << 1) | (((l >> 4) & 1) << 2);
        lanes_of[p] |= 1ull << l;
    }
    for (int ci = 0; ci < 64; ++ci) {
        const int c[3] = {ci & 3, (ci >> 2) & 3, ci >> 4};
        for (int d = 0; d < D; ++d) {
            uint32_t* sl = &slots[((size_t)ci * D + d) * kSlotWords];
            // (offset, weight) of the unmasked entries, and the masked ones with
            // their parity masks; weights carry dx_l / dx_{L-1}
            std::vector<std::pair<uint32_t, double>> plain, masked;
            std::vector<uint32_t> masks;
            {  // dl = 1: configuration = parity of A
                const int combo = (c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1);
                const size_t row = ((size_t)combo * D + d);
                for (int e = 0; e < t.cnt[1][row]; ++e) {
                    const int32_t pk = t.off[1][row * t.len[1] + e];
                    const int o[3] = {(int8_t)(pk & 0xff), (int8_t)((pk >> 8) & 0xff), (int8_t)((pk >> 16) & 0xff)};
                    int u[3];
                    for (int a = 0; a < 3; ++a) u[a] = slot1(c[a] + 4 + o[a]);
                    plain.push_back({(uint32_t)(u[0] + kPy * u[1] + kPz * u[2]), t.w[1][row * t.len[1] + e]});
                }
            }
            {  // dl = 2: configuration = A mod 4
                const int combo = c[0] + 4 * c[1] + 16 * c[2];
                const size_t row = ((size_t)combo * D + d);
                for (int e = 0; e < t.cnt[2][row]; ++e) {
                    const int32_t pk = t.off[2][row * t.len[2] + e];
                    const int o[3] = {(int8_t)(pk & 0xff), (int8_t)((pk >> 8) & 0xff), (int8_t)((pk >> 16) & 0xff)};
                    int u[3];
                    for (int a = 0; a < 3; ++a) u[a] = slot2((c[a] >> 1) + 4 + o[a]);
                    plain.push_back({(uint32_t)(kL2 + u[0] + kPy * u[1] + kPz * u[2]), 2.0 * t.w[2][row * t.len[2] + e]});
                }
            }
            {  // dl = 3: reference fixed by A mod 4; union over the parity of A >> 2
                std::map<int32_t, std::pair<double, int>> uni;  // packed offset -> (w, mask)
                for (int p3 = 0; p3 < 8; ++p3) {
                    int combo = 0, mul = 1;
                    for (int a = 0; a < 3; ++a) {
                        combo += (4 * ((p3 >> a) & 1) + c[a]) * mul;
                        mul *= 8;
                    }
                    const size_t row = ((size_t)combo * D + d);
                    for (int e = 0; e < t.cnt[3][row]; ++e) {
                        const int32_t pk = t.off[3][row * t.len[3] + e];
                        const double wv = t.w[3][row * t.len[3] + e];
                        auto it = uni.find(pk);
                        if (it == uni.end()) {
                            uni[pk] = {wv, 1 << p3};
                        } else {
                            if (std::fabs(it->second.first - wv) > 1e-12) {
                                set_error("internal: dl=3 weights differ across parities");
                                return CD_EINVAL;
                            }
                            it->second.second |= 1 << p3;
                        }
                    }
                }
                for (auto& kv : uni) {
                    const int32_t pk = kv.first;
                    const int o[3] = {(int8_t)(pk & 0xff), (int8_t)((pk >> 8) & 0xff), (int8_t)((pk >> 16) & 0xff)};
                    const uint32_t off = (uint32_t)(kL3 + (5 + o[0]) + kPy * (5 + o[1]) + kPz * (5 + o[2]));
                    if (kv.second.second == 0xff) {
                        plain.push_back({off, 4.0 * kv.second.first});
                    } else {
                        masked.push_back({off, 4.0 * kv.second.first});
                        masks.push_back((uint32_t)kv.second.second);
                    }
                }
            }
            if ((int)plain.size() > kSlotMain + kSlotExtra || (int)masked.size() > kSlotMasked) return CD_OK;
            sl[0] = (uint32_t)plain.size();
            for (size_t e = 0; e < plain.size(); ++e) {
                const bool main = (int)e < kSlotMain;
                const int k = main ? (int)e : (int)e - kSlotMain;
                sl[(main ? kSlotOff : kSlotXOff) + k] = plain[e].first;
                sl[(main ? kSlotW : kSlotXW) + k] = (uint32_t)fbits(plain[e].second);
            }
            for (size_t e = 0; e < masked.size(); ++e) {
                uint64_t lm = 0;
                for (int p = 0; p < 8; ++p)
                    if ((masks[e] >> p) & 1) lm |= lanes_of[p];
                sl[kSlotMOff + e] = masked[e].first;
                sl[kSlotMW + e] = (uint32_t)fbits(masked[e].second);
                sl[kSlotMMask + 2 * e] = (uint32_t)(lm & 0xffffffffu);
                sl[kSlotMMask + 2 * e + 1] = (uint32_t)(lm >> 32);
            }
        }
    }
    t.slots.swap(slots);
    t.tile_ok = true;
    return CD_OK;
}

int build_gather_tables(HostTables& t) {
    const int D = t.D;
    t.ghdr.assign((size_t)64 * D * 4, 0);
    t.gent.clear();
    for (int ci = 0; ci < 64; ++ci) {
        const int c[3] = {ci & 3, (ci >> 2) & 3, ci >> 4};
        for (int d = 0; d < D; ++d) {
            int32_t* h = &t.ghdr[((size_t)ci * D + d) * 4];
            h[0] = (int32_t)(t.gent.size() / 2);
            // dl = 1: configuration = parity of A; dl = 2: A mod 4
            for (int kind = 1; kind <= 2; ++kind) {
                const int combo = kind == 1 ? (c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1) : c[0] + 4 * c[1] + 16 * c[2];
                const size_t row = (size_t)combo * D + d;
                for (int e = 0; e < t.cnt[kind][row]; ++e) {
                    t.gent.push_back(t.off[kind][row * t.len[kind] + e] & 0xffffff);
                    t.gent.push_back(fbits(t.w[kind][row * t.len[kind] + e]));
                }
                h[kind] = t.cnt[kind][row];
            }
            // dl = 3: the reference is fixed by A mod 4, the outer box by the
            // parity p3 of A >> 2: union over p3 with a mask of the parities
            // whose list holds the entry (the chord is the same in all)
            std::map<int32_t, std::pair<double, int>> uni;
            for (int p3 = 0; p3 < 8; ++p3) {
                int combo = 0, mul = 1;
                for (int a = 0; a < 3; ++a) {
                    combo += (4 * ((p3 >> a) & 1) + c[a]) * mul;
                    mul *= 8;
                }
                const size_t row = (size_t)combo * D + d;
                for (int e = 0; e < t.cnt[3][row]; ++e) {
                    const int32_t pk = t.off[3][row * t.len[3] + e] & 0xffffff;
                    const double wv = t.w[3][row * t.len[3] + e];
                    auto it = uni.find(pk);
                    if (it == uni.end()) {
                        uni[pk] = {wv, 1 << p3};
                    } else {
                        if (std::fabs(it->second.first - wv) > 1e-12) {
                            set_error("internal: dl=3 weights differ across parities");
                            return CD_EINVAL;
                        }
                        it->second.second |= 1 << p3;
                    }
                }
            }
            int ncommon = 0, nmasked = 0;
            for (int pass = 0; pass < 2; ++pass)  // entries of every parity first, then the masked ones
                for (auto& kv : uni) {
                    const bool common = kv.second.second == 0xff;
                    if (common != (pass == 0)) continue;
                    t.gent.push_back(kv.first | (common ? 0 : kv.second.second << 24));
                    t.gent.push_back(fbits(kv.second.first));
                    (common ? ncommon : nmasked) += 1;
                }
            h[3] = ncommon | (nmasked << 16);
        }
    }
    t.gent.insert(t.gent.end(), 2 * (size_t)kGatherPad, 0);  // read ahead by the gather (never used)
    return CD_OK;
}

}  // namespace cd

namespace cd {

// Round to bfloat16 / binary16 (nearest, ties to even), as 16-bit patterns.
static uint16_t to_half_bits(double v, int precision) {
    const float f = (float)v;
    if (precision == CD_BF16X2) {
        uint32_t u;
        std::memcpy(&u, &f, 4);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
    const _Float16 h = (_Float16)f;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

static double from_half_bits(uint16_t b, int precision) {
    if (precision == CD_BF16X2) {
        const uint32_t u = (uint32_t)b << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    }
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return (double)(float)h;
}

int build_split_tables(const HostTables& t, int precision, SplitHost& out) {
    using namespace tile;
    const int D = t.D;
    const int nt = (D + 15) / 16;
    const double lo_scale = std::ldexp(1.0, kSplitLoExp[precision]);
    out = SplitHost();
    out.precision = precision;
    out.ntiles = nt;
    out.hdr.assign((size_t)64 * 3 * nt * 2, 0);
    for (int ci = 0; ci < 64; ++ci) {
        const int c[3] = {ci & 3, (ci >> 2) & 3, ci >> 4};
        for (int kind = 1; kind <= 3; ++kind) {
            for (int tl = 0; tl < nt; ++tl) {
                // offset -> (weights of the tile's directions, parity mask)
                std::map<int32_t, std::pair<std::array<double, 16>, int>> uni;
                auto add = [&](int combo, int mask) -> int {
                    for (int j = 0; j < 16 && 16 * tl + j < D; ++j) {
                        const size_t row = (size_t)combo * D + 16 * tl + j;
                        for (int e = 0; e < t.cnt[kind][row]; ++e) {
                            const int32_t pk = t.off[kind][row * t.len[kind] + e];
                            const double wv = t.w[kind][row * t.len[kind] + e];
                            auto it = uni.find(pk);
                            if (it == uni.end()) {
                                std::array<double, 16> z{};
                                it = uni.emplace(pk, std::make_pair(z, 0)).first;
                            }
                            double& slot = it->second.first[j];
                            if (slot != 0.0 && std::fabs(slot - wv) > 1e-12) {
                                set_error("internal: dl=3 weights differ across parities");
                                return CD_EINVAL;
                            }
                            slot = wv;
                            it->second.second |= mask;
                        }
                    }
                    return CD_OK;
                };
                int rc = CD_OK;
                if (kind == 1) rc = add((c[0] & 1) + 2 * (c[1] & 1) + 4 * (c[2] & 1), 0xff);
                else if (kind == 2) rc = add(c[0] + 4 * c[1] + 16 * c[2], 0xff);
                else
                    for (int p3 = 0; p3 < 8 && rc == CD_OK; ++p3) {
                        int combo = 0, mul = 1;
                        for (int a = 0; a < 3; ++a) {
                            combo += (4 * ((p3 >> a) & 1) + c[a]) * mul;
                            mul *= 8;
                        }
                        rc = add(combo, 1 << p3);
                    }
                if (rc != CD_OK) return rc;
                const int n = (int)uni.size();
                const int steps = (n + 31) / 32;
                int32_t* h = &out.hdr[(((size_t)ci * 3 + (kind - 1)) * nt + tl) * 2];
                h[0] = (int32_t)(out.ent.size() / 32);
                h[1] = steps;
                std::vector<int32_t> ent((size_t)steps * 32, 0), eoff((size_t)steps * 32, 0);
                std::vector<std::array<double, 16>> wk((size_t)steps * 32);
                int q = 0;
                for (auto& kv : uni) {
                    const int32_t pk = kv.first;
                    const int o[3] = {(int8_t)(pk & 0xff), (int8_t)((pk >> 8) & 0xff), (int8_t)((pk >> 16) & 0xff)};
                    int u[3];
                    for (int a = 0; a < 3; ++a) {
                        if (kind == 1) {
                            const int v = c[a] + 4 + o[a];
                            u[a] = (v & 3) * 6 + (v >> 2);
                        } else if (kind == 2) {
                            const int v = (c[a] >> 1) + 4 + o[a];
                            u[a] = (v & 1) * 8 + (v >> 1);
                        } else {
                            u[a] = 5 + o[a];
                        }
                    }
                    const int32_t lds = kind == 1   ? u[0] + k1Py * u[1] + k1Pz * u[2]
                                        : kind == 2 ? u[0] + k2Py * u[1] + k2Pz * u[2]
                                                    : u[0] + k3Py * u[1] + k3Pz * u[2];
                    const int mask = kv.second.second;
                    ent[q] = lds | (mask << 16);
                    eoff[q] = (pk & 0xffffff) | (mask << 24);
                    wk[q] = kv.second.first;
                    ++q;
                }
                // padding entries: LDS offset 0, mask 0, weight 0
                out.ent.insert(out.ent.end(), ent.begin(), ent.end());
                out.eoff.insert(out.eoff.end(), eoff.begin(), eoff.end());
                for (int st = 0; st < steps; ++st)
                    for (int L = 0; L < 64; ++L) {
                        const int g = L >> 4, j = L & 15;
                        uint16_t hi8[8], lo8[8];
                        for (int e = 0; e < 8; ++e) {
                            const double K = wk[(size_t)st * 32 + 8 * g + e][j];
                            const uint16_t hb = to_half_bits(K, precision);
                            hi8[e] = hb;
                            lo8[e] = to_half_bits((K - from_half_bits(hb, precision)) * lo_scale, precision);
                        }
                        out.bank.insert(out.bank.end(), hi8, hi8 + 8);
                        out.bank.insert(out.bank.end(), lo8, lo8 + 8);
                    }
            }
        }
    }
    return CD_OK;
}

}  // namespace cd
