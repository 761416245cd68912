// Gas heating driven by the screening factor (Sect. 5): the Draine field G0
// attenuated by chi, G0_eff = chi G0; photoelectric heating on small grains
// and PAHs, Gamma_UV = 1e-24 eps G0_eff n, with the efficiency of Wolfire et
// al. (1995) in x = G0_eff T^(1/2) / n_e,
//   eps = 4.9e-2 / (1 + (x / 1925)^0.73) + 3.7e-2 (T / 1e4)^0.7 / (1 + x / 5000);
// cosmic-ray heating Gamma_CR = 1e-27 n (erg cm^-3 s^-1).  One thread per
// cell; chi either given or, fused, averaged from the cell's row of N (Eq. 7).
#include <cmath>

#include "cd_internal.h"

namespace cd {

struct HeatArgs {
    const float* N;     // [n][D] columns, or nullptr: chi is an input
    int D;
    float chi_scale;    // gamma av_per_nh
    const float* n;     // hydrogen density
    const float* T;
    const float* ne;
    float G0;
    const float* chi_in;
    float* chi_out;     // may be nullptr
    float* g0eff;       // may be nullptr
    float* uv;
    float* cr;          // may be nullptr
    int64_t cells;
};

__global__ __launch_bounds__(256) void k_heating(const HeatArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.cells) return;
    float chi;
    if (a.N) {
        const float* row = a.N + i * a.D;
        float s = 0.f;
        for (int d = 0; d < a.D; ++d) s += expf(-a.chi_scale * row[d]);
        chi = s / (float)a.D;
        if (a.chi_out) a.chi_out[i] = chi;
    } else {
        chi = a.chi_in[i];
    }
    const float n = a.n[i], T = a.T[i], ne = a.ne[i];
    const float g = chi * a.G0;
    const float gt = g * sqrtf(T);
    const float x = ne > 0.f ? gt / ne : (gt > 0.f ? INFINITY : 0.f);
    const float eps = 4.9e-2f / (1.f + powf(x * (1.f / 1925.f), 0.73f)) +
                      3.7e-2f * powf(T * 1e-4f, 0.7f) / (1.f + x * (1.f / 5000.f));
    if (a.g0eff) a.g0eff[i] = g;
    a.uv[i] = 1e-24f * eps * g * n;
    if (a.cr) a.cr[i] = 1e-27f * n;
}

static int launch_heating(const HeatArgs& a, hipStream_t s) {
    if (a.cells == 0) return CD_OK;
    k_heating<<<(unsigned)((a.cells + 255) / 256), 256, 0, s>>>(a);
    CD_HIP(hipGetLastError());
    return CD_OK;
}

}  // namespace cd

extern "C" int cd_heating_rates(const float* chi_dev, const float* n_dev, const float* T_dev, const float* ne_dev,
                                int64_t n_cells, double G0, float* g0eff_dev, float* gamma_uv_dev,
                                float* gamma_cr_dev, void* stream) {
    cd::clear_error();
    if (n_cells < 0 || (n_cells > 0 && (!chi_dev || !n_dev || !T_dev || !ne_dev || !gamma_uv_dev)) ||
        !std::isfinite(G0) || G0 < 0) {
        cd::set_error("cd_heating_rates: NULL buffer, n_cells %lld < 0 or G0 %g", (long long)n_cells, G0);
        return CD_EINVAL;
    }
    cd::HeatArgs a{};
    a.n = n_dev;
    a.T = T_dev;
    a.ne = ne_dev;
    a.G0 = (float)G0;
    a.chi_in = chi_dev;
    a.g0eff = g0eff_dev;
    a.uv = gamma_uv_dev;
    a.cr = gamma_cr_dev;
    a.cells = n_cells;
    return cd::launch_heating(a, (hipStream_t)stream);
}

extern "C" int cd_screening_heating(const float* N_dev, int64_t n_cells, int D, double av_per_nh, double gamma,
                                    const float* n_dev, const float* T_dev, const float* ne_dev, double G0,
                                    float* chi_dev, float* g0eff_dev, float* gamma_uv_dev, float* gamma_cr_dev,
                                    void* stream) {
    cd::clear_error();
    if (n_cells < 0 || D < 1 || D > CD_MAX_DIRS ||
        (n_cells > 0 && (!N_dev || !n_dev || !T_dev || !ne_dev || !gamma_uv_dev)) || !std::isfinite(G0) || G0 < 0 ||
        !std::isfinite(av_per_nh) || !std::isfinite(gamma)) {
        cd::set_error("cd_screening_heating: NULL buffer, n_cells %lld, D %d or a non-finite parameter",
                      (long long)n_cells, D);
        return CD_EINVAL;
    }
    cd::HeatArgs a{};
    a.N = N_dev;
    a.D = D;
    a.chi_scale = (float)(gamma * av_per_nh);
    a.n = n_dev;
    a.T = T_dev;
    a.ne = ne_dev;
    a.G0 = (float)G0;
    a.chi_out = chi_dev;
    a.g0eff = g0eff_dev;
    a.uv = gamma_uv_dev;
    a.cr = gamma_cr_dev;
    a.cells = n_cells;
    return cd::launch_heating(a, (hipStream_t)stream);
}
