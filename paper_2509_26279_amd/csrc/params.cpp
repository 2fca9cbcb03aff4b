// Threshold rule of Sec. 2.2 (Setting the algorithm parameters).
//
// The number of noise detections in a bin is Poisson; with mu noise
// detections per bin per epoch, a bin holds a noise detection in a given
// epoch with probability p = 1 - exp(-mu), so the distinct epochs of a
// pure-noise bin are Binomial(E, p) and its detections Poisson(E mu).  N_min
// is the smallest count whose tail probability, times the number of
// independent stacks (eq. N_stacks), is at most the admissible number of
// false results.
#include <cmath>
#include <string>

#include "internal.h"

namespace sas {
void set_error(const std::string &msg);
}

namespace {

// P(X >= k) for X ~ Binomial(n, p), summed from the top in long double.
long double binom_tail(int k, int n, long double p) {
    if (k <= 0) return 1.0L;
    if (k > n) return 0.0L;
    if (p <= 0.0L) return 0.0L;
    if (p >= 1.0L) return 1.0L;
    const long double lp = std::log(p), lq = std::log1p(-p);
    long double s = 0.0L;
    for (int i = n; i >= k; --i) {
        const long double lc = std::lgamma((long double)n + 1) - std::lgamma((long double)i + 1) -
                               std::lgamma((long double)(n - i) + 1);
        s += std::exp(lc + i * lp + (n - i) * lq);
    }
    return s;
}

// P(X >= k) for X ~ Poisson(lam): one minus the lower sum, or the upper
// sum directly when the lower sum is close to one.
long double poisson_tail(int k, long double lam) {
    if (k <= 0) return 1.0L;
    if (lam <= 0.0L) return 0.0L;
    long double term = std::exp(-lam), lower = 0.0L;
    for (int i = 0; i < k; ++i) {
        lower += term;
        term *= lam / (i + 1);
    }
    if (lower < 0.5L) return 1.0L - lower;
    long double upper = 0.0L;  // term is now P(X = k)
    for (int i = k; i < k + 100000; ++i) {
        upper += term;
        term *= lam / (i + 1);
        if (term < upper * 1e-22L) break;
    }
    return upper;
}

}  // namespace

extern "C" sas_status sas_threshold_n_min(int32_t n_epochs, double mu, double n_stacks,
                                          double n_false, int32_t mode, int32_t *n_min_out) {
    if (!n_min_out || n_epochs < 1 || !(mu >= 0.0) || !(n_stacks >= 0.0) || !(n_false > 0.0) ||
        (mode != SAS_MODE_EPOCHS && mode != SAS_MODE_DETECTIONS)) {
        sas::set_error("sas_threshold_n_min: bad argument");
        return SAS_E_INVALID;
    }
    const long double p = -std::expm1(-(long double)mu);
    for (int n = 1; n < 1000000; ++n) {
        const long double tail = mode == SAS_MODE_EPOCHS
                                     ? binom_tail(n, n_epochs, p)
                                     : poisson_tail(n, (long double)n_epochs * mu);
        if ((long double)n_stacks * tail <= (long double)n_false) {
            *n_min_out = n;
            return SAS_OK;
        }
        if (mode == SAS_MODE_EPOCHS && n > n_epochs) break;
    }
    sas::set_error("sas_threshold_n_min: no threshold reaches the requested false-result count");
    return SAS_E_INVALID;
}
