// muca_analysis.cpp -- production analysis on the host (include/muca.h,
// muca_jackknife_log_dos and muca_canonical).
//
// A production run at fixed weights omega, cut into B calls, gives B block
// histograms H_b (Sec. 3.3: the paper uses 100 calls).  The estimate of the
// density of states is ln g = ln H - omega (+ const) from the summed histogram
// (Sec. 2.1); its error bars come from a jackknife over the blocks: the same
// estimate from the sum without block b, for every b.  Canonical averages at
// inverse temperature beta follow by reweighting, <O>_beta = sum_E g(E)
// e^{-beta E} O(E) / Z_beta (Sec. 2.1), all in logarithms to avoid overflow.
#include <algorithm>
#include <cmath>
#include <limits>
#include <new>
#include <vector>

#include "muca.h"
#include "muca_host_math.h"

namespace {

constexpr double kNaN = std::numeric_limits<double>::quiet_NaN();

bool log_dos(uint32_t N, const uint64_t* H, const double* omega, int normalization, double* out)
{
    return muca_host::log_dos_of(N, H, omega, normalization, out) == 0;
}

// Canonical mean energy per spin and specific heat per spin at beta from
// ln g (energies E_k = 4k - 2N).
void canonical_one(uint32_t N, const double* lng, double beta, double* e, double* c)
{
    double mx = -INFINITY;
    for (uint32_t k = 0; k <= N; ++k)
        if (lng[k] != -INFINITY)
            mx = std::max(mx, lng[k] - beta * (4.0 * k - 2.0 * N));
    double z = 0.0, s1 = 0.0, s2 = 0.0;
    for (uint32_t k = 0; k <= N; ++k) {
        if (lng[k] == -INFINITY)
            continue;
        const double E = 4.0 * k - 2.0 * N;
        const double p = std::exp(lng[k] - beta * E - mx);
        z += p;
        s1 += p * E;
        s2 += p * E * E;
    }
    const double m1 = s1 / z, m2 = s2 / z;
    *e = m1 / N;
    *c = beta * beta * (m2 - m1 * m1) / N;
}

bool args_ok(uint32_t L, uint32_t blocks, const uint64_t* h, const double* omega)
{
    return L >= 4 && L <= MUCA_MAX_L && L % 2 == 0 && blocks >= 1 && h && omega;
}

// Jackknife error of a statistic from its B leave-one-out values.
double jk_error(const std::vector<double>& loo)
{
    const size_t B = loo.size();
    if (B < 2)
        return 0.0;
    double mean = 0.0;
    for (double v : loo)
        mean += v;
    mean /= (double)B;
    double ss = 0.0;
    for (double v : loo)
        ss += (v - mean) * (v - mean);
    return std::sqrt((double)(B - 1) / (double)B * ss);
}

}  // namespace

extern "C" {

static int muca_jackknife_log_dos_impl(uint32_t L, uint32_t blocks, const uint64_t* block_hists,
                                       const double* omega, int normalization, double* ln_g, double* ln_g_err)
{
    if (!args_ok(L, blocks, block_hists, omega) || !ln_g || (normalization != 0 && normalization != 1))
        return MUCA_ERR_INVALID_ARG;
    const uint32_t N = L * L, nb = N + 1;
    std::vector<uint64_t> total(nb, 0), loo_h(nb);
    for (uint32_t b = 0; b < blocks; ++b)
        for (uint32_t k = 0; k < nb; ++k)
            total[k] += block_hists[(size_t)b * nb + k];
    if (!log_dos(N, total.data(), omega, normalization, ln_g))
        return MUCA_ERR_NOT_CONVERGED;
    if (!ln_g_err)
        return MUCA_OK;
    std::vector<std::vector<double>> loo(nb, std::vector<double>(blocks));
    std::vector<double> est(nb);
    std::vector<bool> broken(nb, false);
    for (uint32_t b = 0; b < blocks; ++b) {
        for (uint32_t k = 0; k < nb; ++k)
            loo_h[k] = total[k] - block_hists[(size_t)b * nb + k];
        if (blocks > 1 && !log_dos(N, loo_h.data(), omega, normalization, est.data())) {
            std::fill(broken.begin(), broken.end(), true);
            continue;
        }
        for (uint32_t k = 0; k < nb; ++k) {
            if (blocks > 1 && (est[k] == -INFINITY) != (ln_g[k] == -INFINITY))
                broken[k] = true;  // the bin is empty without block b
            loo[k][b] = blocks > 1 ? est[k] : ln_g[k];
        }
    }
    for (uint32_t k = 0; k < nb; ++k) {
        if (ln_g[k] == -INFINITY)
            ln_g_err[k] = kNaN;
        else if (broken[k])
            ln_g_err[k] = INFINITY;
        else
            ln_g_err[k] = jk_error(loo[k]);
    }
    return MUCA_OK;
}

// No C++ exception leaves the C ABI: a failed host allocation is reported.
int muca_jackknife_log_dos(uint32_t L, uint32_t blocks, const uint64_t* block_hists,
                           const double* omega, int normalization, double* ln_g, double* ln_g_err)
{
    try {
        return muca_jackknife_log_dos_impl(L, blocks, block_hists, omega, normalization, ln_g, ln_g_err);
    } catch (const std::bad_alloc&) {
        return MUCA_ERR_OUT_OF_MEMORY;
    } catch (...) {
        return MUCA_ERR_STATE;
    }
}

static int muca_canonical_impl(uint32_t L, uint32_t blocks, const uint64_t* block_hists, const double* omega,
                               uint32_t n_beta, const double* betas, double* energy, double* energy_err,
                               double* specific_heat, double* specific_heat_err)
{
    if (!args_ok(L, blocks, block_hists, omega) || (n_beta && (!betas || !energy || !specific_heat)))
        return MUCA_ERR_INVALID_ARG;
    const uint32_t N = L * L, nb = N + 1;
    std::vector<uint64_t> total(nb, 0), loo_h(nb);
    for (uint32_t b = 0; b < blocks; ++b)
        for (uint32_t k = 0; k < nb; ++k)
            total[k] += block_hists[(size_t)b * nb + k];
    std::vector<double> lng(nb);
    // the normalisation cancels in canonical averages; the sum form needs no anchor bin
    if (!log_dos(N, total.data(), omega, 1, lng.data()))
        return MUCA_ERR_NOT_CONVERGED;
    for (uint32_t j = 0; j < n_beta; ++j)
        canonical_one(N, lng.data(), betas[j], &energy[j], &specific_heat[j]);
    if (!energy_err && !specific_heat_err)
        return MUCA_OK;
    std::vector<std::vector<double>> le(n_beta, std::vector<double>(blocks)),
        lc(n_beta, std::vector<double>(blocks));
    bool broken = false;
    for (uint32_t b = 0; b < blocks && blocks > 1; ++b) {
        for (uint32_t k = 0; k < nb; ++k)
            loo_h[k] = total[k] - block_hists[(size_t)b * nb + k];
        if (!log_dos(N, loo_h.data(), omega, 1, lng.data())) {
            broken = true;
            break;
        }
        for (uint32_t j = 0; j < n_beta; ++j)
            canonical_one(N, lng.data(), betas[j], &le[j][b], &lc[j][b]);
    }
    for (uint32_t j = 0; j < n_beta; ++j) {
        const double ee = blocks > 1 ? (broken ? INFINITY : jk_error(le[j])) : 0.0;
        const double ce = blocks > 1 ? (broken ? INFINITY : jk_error(lc[j])) : 0.0;
        if (energy_err)
            energy_err[j] = ee;
        if (specific_heat_err)
            specific_heat_err[j] = ce;
    }
    return MUCA_OK;
}

// No C++ exception leaves the C ABI: a failed host allocation is reported.
int muca_canonical(uint32_t L, uint32_t blocks, const uint64_t* block_hists, const double* omega,
                   uint32_t n_beta, const double* betas, double* energy, double* energy_err,
                   double* specific_heat, double* specific_heat_err)
{
    try {
        return muca_canonical_impl(L, blocks, block_hists, omega, n_beta, betas, energy, energy_err, specific_heat,
                                   specific_heat_err);
    } catch (const std::bad_alloc&) {
        return MUCA_ERR_OUT_OF_MEMORY;
    } catch (...) {
        return MUCA_ERR_STATE;
    }
}

}  // extern "C"
