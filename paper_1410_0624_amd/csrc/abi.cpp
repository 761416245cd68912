// Error reporting, directions and weight upload of the colden C ABI.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cd_internal.h"

namespace cd {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

void* DevArena::take(size_t bytes, bool* ok) {
    const size_t off = (used + 255) & ~(size_t)255;
    used = off + bytes;
    if (!base) return nullptr;
    if (used > cap) {
        if (*ok) set_error("workspace of %zu bytes is too small (the workspace-size query gives what is needed)", cap);
        *ok = false;
        return nullptr;
    }
    return base + off;
}

}  // namespace cd

extern "C" const char* cd_last_error(void) { return cd::g_err; }

extern "C" int cd_version(void) { return 2; }

extern "C" int cd_directions(int scheme, int p1, int p2, double* out, int capacity, int* D) {
    cd::clear_error();
    if (!D || (!out && capacity > 0)) {
        cd::set_error("cd_directions: NULL output");
        return CD_EINVAL;
    }
    std::vector<std::array<double, 3>> v;
    int rc = cd::make_directions(scheme, p1, p2, v);
    if (rc != CD_OK) {
        cd::set_error("cd_directions: bad scheme %d or parameters (%d, %d)", scheme, p1, p2);
        return rc;
    }
    if ((int)v.size() > capacity) {
        cd::set_error("cd_directions: capacity %d < %zu directions", capacity, v.size());
        *D = (int)v.size();
        return CD_EINVAL;
    }
    for (size_t d = 0; d < v.size(); ++d)
        for (int k = 0; k < 3; ++k) out[3 * d + k] = v[d][k];
    *D = (int)v.size();
    return CD_OK;
}

namespace cd {
int upload_split_banks(cd_weights* w, hipStream_t s);  // split.hip
}

// Directions as unit vectors (finite, |u| = 1 within 1e-9).
static bool unit_dirs(const char* who, const double* dirs, int D, std::vector<std::array<double, 3>>& u) {
    u.assign(D, {0.0, 0.0, 0.0});
    for (int d = 0; d < D; ++d) {
        double n2 = 0;
        for (int k = 0; k < 3; ++k) {
            u[d][k] = dirs[3 * d + k];
            if (!std::isfinite(u[d][k])) {
                cd::set_error("%s: direction %d is not finite", who, d);
                return false;
            }
            n2 += u[d][k] * u[d][k];
        }
        if (std::fabs(std::sqrt(n2) - 1.0) > 1e-9) {
            cd::set_error("%s: direction %d is not a unit vector", who, d);
            return false;
        }
    }
    return true;
}

// The weight tables of one direction set (FP64 on the host, Sect. 3.3) and
// their copies in the workspace: FP32 lists, tile slots, gather tables and
// split banks.  With w->ws in a sizing pass only the bytes are counted.
static int weights_build(const std::vector<std::array<double, 3>>& u, cd_weights* w, hipStream_t s) {
    const int D = w->D;
    int rc = cd::build_tables(u, w->host);
    if (rc == CD_OK) rc = cd::build_tile_tables(u, w->host);
    if (rc == CD_OK) rc = cd::build_gather_tables(w->host);
    if (rc != CD_OK) return rc;
    // host staging buffers live until the stream is synchronised by the caller
    std::vector<std::vector<float>> wf(cd::kKinds), wtf(cd::kKinds);
    std::vector<std::vector<int32_t>> otf(cd::kKinds);
    for (int k = 1; k < cd::kKinds && rc == CD_OK; ++k) {
        w->ncombo[k] = w->host.ncombo[k];
        w->len[k] = w->host.len[k];
        wf[k].assign(w->host.w[k].begin(), w->host.w[k].end());
        rc = cd::ws_upload(w->ws, w->host.off[k], &w->off[k], s);
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, wf[k], &w->w[k], s);
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, w->host.cnt[k], &w->cnt[k], s);
        // the same lists with the direction fastest, for kernels with a lane per direction
        const size_t nc = (size_t)w->ncombo[k], len = (size_t)w->len[k];
        otf[k].assign(nc * len * D, 0);
        wtf[k].assign(nc * len * D, 0.f);
        for (size_t c = 0; c < nc; ++c)
            for (size_t d = 0; d < (size_t)D; ++d)
                for (size_t e = 0; e < len; ++e) {
                    otf[k][(c * len + e) * D + d] = w->host.off[k][(c * D + d) * len + e];
                    wtf[k][(c * len + e) * D + d] = (float)w->host.w[k][(c * D + d) * len + e];
                }
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, otf[k], &w->offT[k], s);
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, wtf[k], &w->wT[k], s);
    }
    {
        // kind-4 offsets (x, y, z bytes) as word offsets in the coarse-table
        // kernel's cell window (pitches kCellWinPy, kCellWinPz)
        const std::vector<int32_t>& o4 = w->host.off[4];
        std::vector<int32_t> ow(o4.size());
        for (size_t i = 0; i < o4.size(); ++i) {
            const int sx = (int8_t)(o4[i] & 0xff), sy = (int8_t)((o4[i] >> 8) & 0xff), sz = (int8_t)((o4[i] >> 16) & 0xff);
            ow[i] = sz * cd::kCellWinPz + sy * cd::kCellWinPy + sx;
        }
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, ow, &w->offwin4, s);
    }
    std::vector<float> kf(w->host.kloc.begin(), w->host.kloc.end());
    std::vector<float> gf(w->host.gloc.begin(), w->host.gloc.end());
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, kf, &w->kloc, s);
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, w->host.slots, &w->slots, s);
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, gf, &w->gloc, s);
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, w->host.sgn, &w->sgn, s);
    {
        // the row kernel's chords per direction and parity (oy, oz) of the
        // target row: for the pair of x targets of an oct, own-column chords
        // Wo[j] and sibling-column chords of the low (Wsl) and high (Wsh)
        // target, zero where the ray cannot cross into that sibling
        const int D = w->D;
        std::vector<float> gq((size_t)D * 4 * 12, 0.f);
        for (int d = 0; d < D; ++d) {
            const int sg = w->host.sgn[(size_t)d];
            const bool fx0 = (sg & 1) == 0;  // the low-x target runs into its x sibling
            for (int q = 0; q < 4; ++q) {
                const int oy = q & 1, oz = q >> 1;
                const int fyz = (oy == ((sg >> 1) & 1) ? 1 : 0) | (oz == ((sg >> 2) & 1) ? 2 : 0);
                float* g = &gq[((size_t)d * 4 + q) * 12];
                for (int j = 0; j < 4; ++j) {
                    if ((j & fyz) != j) continue;
                    g[j] = (float)w->host.gloc[(size_t)d * 8 + 2 * j];
                    const float sib = (float)w->host.gloc[(size_t)d * 8 + 2 * j + 1];
                    (fx0 ? g[4 + j] : g[8 + j]) = sib;
                }
            }
        }
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, gq, &w->glq, s);
        // the same chords as the matrix of the row kernel's matrix-core form:
        // row c = cx + 2 cy + 4 cz (the oct's cell), column x D + d (the x
        // target of the pair, direction), per row parity; columns padded to
        // a multiple of 16 with zeros
        const int nc = 16 * ((2 * D + 15) / 16);
        std::vector<float> gm((size_t)4 * 8 * nc, 0.f);
        for (int q = 0; q < 4; ++q) {
            const int oy = q & 1, oz = q >> 1;
            for (int c = 0; c < 8; ++c) {
                const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
                const int j = (cy ^ oy) + 2 * (cz ^ oz);
                for (int x = 0; x < 2; ++x)
                    for (int d = 0; d < D; ++d) {
                        const float* g = &gq[((size_t)d * 4 + q) * 12];
                        gm[((size_t)q * 8 + c) * nc + x * D + d] = cx == x ? g[j] : g[(x == 0 ? 4 : 8) + j];
                    }
            }
        }
        if (rc == CD_OK) rc = cd::ws_upload(w->ws, gm, &w->glm, s);
    }
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, w->host.ghdr, &w->ghdr, s);
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, w->host.gent, &w->gent, s);
    // [D][6]: the unit vector (components below 1e-14 snapped to 0) and the
    // reciprocals of its components (0 where a component is 0)
    std::vector<double> du((size_t)D * 6);
    for (int d = 0; d < D; ++d)
        for (int k = 0; k < 3; ++k) {
            const double c = std::fabs(u[d][k]) < 1e-14 ? 0.0 : u[d][k];
            du[(size_t)d * 6 + k] = c;
            du[(size_t)d * 6 + 3 + k] = c != 0.0 ? 1.0 / c : 0.0;
        }
    if (rc == CD_OK) rc = cd::ws_upload(w->ws, du, &w->dirs, s);
    if (rc == CD_OK && w->precision != CD_FP32) rc = cd::upload_split_banks(w, s);
    if (rc == CD_OK && !w->ws.sizing() && hipStreamSynchronize(s) != hipSuccess) {
        cd::set_error("cd_precompute_weights: upload failed");
        rc = CD_EDEVICE;
    }
    return rc;
}

static int weights_args(const char* who, const double* dirs, int D, int mode, int precision,
                        std::vector<std::array<double, 3>>& u) {
    if (D < 1 || D > CD_MAX_DIRS) {
        cd::set_error("%s: D = %d outside 1..%d", who, D, CD_MAX_DIRS);
        return CD_EINVAL;
    }
    if (mode != CD_PRECALC73 && mode != CD_INSITU) {
        cd::set_error("%s: unknown mode %d", who, mode);
        return CD_EINVAL;
    }
    if (precision != CD_FP32 && precision != CD_BF16X2 && precision != CD_FP16X2) {
        cd::set_error("%s: unknown precision %d", who, precision);
        return CD_EINVAL;
    }
    return unit_dirs(who, dirs, D, u) ? CD_OK : CD_EINVAL;
}

extern "C" int cd_weights_workspace_bytes(const double* dirs, int D, int mode, int precision, size_t* bytes) {
    cd::clear_error();
    if (!dirs || !bytes) {
        cd::set_error("cd_weights_workspace_bytes: NULL argument");
        return CD_EINVAL;
    }
    std::vector<std::array<double, 3>> u;
    int rc = weights_args("cd_weights_workspace_bytes", dirs, D, mode, precision, u);
    if (rc != CD_OK) return rc;
    cd_weights w;
    w.D = D;
    w.mode = mode;
    w.precision = precision;
    rc = weights_build(u, &w, nullptr);  // sizing pass: no device access
    if (rc == CD_OK) *bytes = w.ws.used;
    return rc;
}

extern "C" int cd_precompute_weights(const double* dirs, int D, int mode, int precision, void* workspace_dev,
                                     size_t workspace_bytes, void* stream, cd_weights** out) {
    cd::clear_error();
    if (!dirs || !out || !workspace_dev) {
        cd::set_error("cd_precompute_weights: NULL argument");
        return CD_EINVAL;
    }
    *out = nullptr;
    if (!cd::is_aligned(workspace_dev, 256)) {
        cd::set_error("cd_precompute_weights: the workspace must be 256-byte aligned");
        return CD_EINVAL;
    }
    std::vector<std::array<double, 3>> u;
    int rc = weights_args("cd_precompute_weights", dirs, D, mode, precision, u);
    if (rc != CD_OK) return rc;
    cd_weights* w = new cd_weights();
    w->D = D;
    w->mode = mode;
    w->precision = precision;
    w->ws.base = static_cast<char*>(workspace_dev);
    w->ws.cap = workspace_bytes;
    rc = weights_build(u, w, (hipStream_t)stream);
    if (rc != CD_OK) {
        // the copies already issued read host vectors that end here
        (void)hipStreamSynchronize((hipStream_t)stream);
        delete w;
        return rc;
    }
    *out = w;
    return CD_OK;
}

extern "C" int cd_weight_lists(const double* dirs, int D, int kind, int* ncombo, int* len, int32_t* off,
                               double* w, int32_t* cnt, double* ref, int32_t* box) {
    cd::clear_error();
    if (!dirs || !ncombo || !len || D < 1 || D > CD_MAX_DIRS || kind < 0 || kind > 4) {
        cd::set_error("cd_weight_lists: bad arguments (D %d, kind %d)", D, kind);
        return CD_EINVAL;
    }
    std::vector<std::array<double, 3>> u;
    if (!unit_dirs("cd_weight_lists", dirs, D, u)) return CD_EINVAL;
    cd::HostTables t;
    int rc = cd::build_tables(u, t);
    if (rc != CD_OK) return rc;
    if (kind == 0) {
        // internal + local: combo = octant a of the target in its oct, the 8
        // oct cells s = i + 2j + 4k as entries
        *ncombo = 8;
        *len = 8;
        if (!off) return CD_OK;
        for (int a = 0; a < 8; ++a) {
            if (ref)
                for (int k = 0; k < 3; ++k) ref[3 * a + k] = ((a >> k) & 1) + 0.5;
            for (int d = 0; d < D; ++d) {
                if (cnt) cnt[a * D + d] = 8;
                for (int s8 = 0; s8 < 8; ++s8) {
                    const size_t e = ((size_t)a * D + d) * 8 + s8;
                    for (int k = 0; k < 3; ++k) off[3 * e + k] = (s8 >> k) & 1;
                    if (w) w[e] = t.kloc[((size_t)a * 8 + s8) * D + d];
                }
            }
        }
        return CD_OK;
    }
    const std::vector<cd::AxisShape> sh = cd::axis_shapes(kind);
    const int na = (int)sh.size();
    *ncombo = t.ncombo[kind];
    *len = t.len[kind];
    if (!off) return CD_OK;
    const size_t L = (size_t)t.len[kind];
    for (int c = 0; c < t.ncombo[kind]; ++c) {
        const cd::AxisShape* a[3] = {&sh[c % na], &sh[(c / na) % na], &sh[c / (na * na)]};
        for (int k = 0; k < 3; ++k) {
            if (ref) ref[3 * c + k] = a[k]->ref;
            if (box) {
                box[12 * c + 4 * k] = a[k]->ilo;
                box[12 * c + 4 * k + 1] = a[k]->ihi;
                box[12 * c + 4 * k + 2] = a[k]->olo;
                box[12 * c + 4 * k + 3] = a[k]->ohi;
            }
        }
        for (int d = 0; d < D; ++d) {
            const size_t q = (size_t)c * D + d;
            if (cnt) cnt[q] = t.cnt[kind][q];
            for (size_t e = 0; e < L; ++e) {
                const int32_t pk = t.off[kind][q * L + e];
                off[3 * (q * L + e)] = (int8_t)(pk & 0xff);
                off[3 * (q * L + e) + 1] = (int8_t)((pk >> 8) & 0xff);
                off[3 * (q * L + e) + 2] = (int8_t)((pk >> 16) & 0xff);
                if (w) w[q * L + e] = t.w[kind][q * L + e];
            }
        }
    }
    return CD_OK;
}

extern "C" int cd_weights_n_dirs(const cd_weights* w, int* D) {
    if (!w || !D) {
        cd::set_error("cd_weights_n_dirs: NULL argument");
        return CD_EINVAL;
    }
    *D = w->D;
    return CD_OK;
}

extern "C" int cd_weights_split_steps(const cd_weights* w, int64_t* steps) {
    if (!w || !steps) {
        cd::set_error("cd_weights_split_steps: NULL argument");
        return CD_EINVAL;
    }
    int64_t n = 0;
    const std::vector<int32_t>& h = w->split_host.hdr;
    for (size_t i = 1; i < h.size(); i += 2) n += h[i];
    *steps = n;
    return CD_OK;
}

extern "C" void cd_weights_destroy(cd_weights* w) {
    delete w;  // its device memory is the caller's workspace
}
