// Reference-parameter search (Sec. II C): CMA-ES over the full-band likelihood.
//
// The population's fitness is the full-band lnL of Eqs. (2)-(3) (with the Planck taper of
// IMRPhenomD_NRTidalv2), evaluated on the device for the whole population at once; the
// strategy's update -- a few hundred operations on 13-vectors and a 13 x 13 covariance -- runs
// on the host between two evaluations.  Hansen's (mu/mu_w, lambda)-CMA-ES with cumulative
// step-size adaptation and the default constants, maximising, in box-normalised coordinates
// u = (theta - lo) / (hi - lo); candidates are x = m + sigma A z with A the lower Cholesky
// factor of C, and the step-size path uses A^{-1} <y>_w.  A candidate outside the box ranks
// below every candidate inside it; equal fitness keeps the candidates' order.  A run ends
// early once its covariance is too ill-conditioned to factor reliably.
//
// Several independent runs from the caller's starting points (a multistart: the likelihood
// surface of a long inspiral has many separated local maxima along the chirp-mass / time
// ridge and over the sky, and one run ends in whichever it meets first) advance together:
// each generation evaluates the populations of all running runs in one batch on the device,
// and the best candidate over all runs is returned.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "rbl_host.h"

using namespace rbl;

namespace {

constexpr int kN = 13;

struct Cmaes {
    int lam, mu;
    std::vector<double> w;
    double mueff, cc, cs, c1, cmu, ds, chi_n;
    double m[kN], ps[kN] = {}, pc[kN] = {}, C[kN][kN] = {}, A[kN][kN] = {};
    double sigma;
    int64_t gen = 0;

    Cmaes(const double* m0, double sigma0, int lambda) : lam(lambda), mu(lambda / 2), sigma(sigma0) {
        const double n = kN;
        w.resize((size_t)mu);
        double s = 0.0;
        for (int i = 0; i < mu; ++i) s += (w[(size_t)i] = std::log(mu + 0.5) - std::log(i + 1.0));
        double s2 = 0.0;
        for (double& x : w) {
            x /= s;
            s2 += x * x;
        }
        mueff = 1.0 / s2;
        cc = (4.0 + mueff / n) / (n + 4.0 + 2.0 * mueff / n);
        cs = (mueff + 2.0) / (n + mueff + 5.0);
        c1 = 2.0 / ((n + 1.3) * (n + 1.3) + mueff);
        cmu = std::min(1.0 - c1, 2.0 * (mueff - 2.0 + 1.0 / mueff) / ((n + 2.0) * (n + 2.0) + mueff));
        ds = 1.0 + 2.0 * std::max(0.0, std::sqrt((mueff - 1.0) / (n + 1.0)) - 1.0) + cs;
        chi_n = std::sqrt(n) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n));
        for (int i = 0; i < kN; ++i) {
            m[i] = m0[i];
            C[i][i] = 1.0;
        }
    }

    // Lower Cholesky factor A of C; false when the search must stop: C not positive definite
    // in floating point, (max_i A_ii / min_i A_ii)^2 -- a lower bound of its condition number --
    // above 1e14, or the largest step sigma max_i A_ii beyond the box width (the ConditionCov
    // and TolUpSigma termination criteria of the CMA-ES tutorial, on the Cholesky factor).
    bool factor() {
        for (int i = 0; i < kN; ++i)
            for (int j = 0; j <= i; ++j) {
                double s = C[i][j];
                for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
                if (i == j) {
                    if (!(s > 0.0)) return false;
                    A[i][i] = std::sqrt(s);
                } else {
                    A[i][j] = s / A[j][j];
                }
            }
        for (int i = 0; i < kN; ++i)
            for (int j = i + 1; j < kN; ++j) A[i][j] = 0.0;
        double dmax = A[0][0], dmin = A[0][0];
        for (int i = 1; i < kN; ++i) {
            dmax = std::max(dmax, A[i][i]);
            dmin = std::min(dmin, A[i][i]);
        }
        return (dmax / dmin) * (dmax / dmin) <= 1e14 && sigma * dmax <= 1.0;
    }

    // y = A z for one candidate.
    void sample(const double* z, double* y) const {
        for (int i = 0; i < kN; ++i) {
            double s = 0.0;
            for (int k = 0; k <= i; ++k) s += A[i][k] * z[k];
            y[i] = s;
        }
    }

    // Update from the candidates' steps y [lam][kN] and fitness [lam] (larger is better).
    void tell(const double* y, const double* fit) {
        std::vector<int> order((size_t)lam);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fit[a] > fit[b]; });
        double yw[kN] = {};
        for (int i = 0; i < mu; ++i)
            for (int k = 0; k < kN; ++k) yw[k] += w[(size_t)i] * y[(size_t)order[(size_t)i] * kN + k];
        for (int k = 0; k < kN; ++k) m[k] += sigma * yw[k];
        double zw[kN];  // A^{-1} yw by forward substitution
        for (int i = 0; i < kN; ++i) {
            double s = yw[i];
            for (int k = 0; k < i; ++k) s -= A[i][k] * zw[k];
            zw[i] = s / A[i][i];
        }
        const double a_s = std::sqrt(cs * (2.0 - cs) * mueff);
        double nps = 0.0;
        for (int k = 0; k < kN; ++k) {
            ps[k] = (1.0 - cs) * ps[k] + a_s * zw[k];
            nps += ps[k] * ps[k];
        }
        nps = std::sqrt(nps);
        ++gen;
        const bool hs = nps / std::sqrt(1.0 - std::pow(1.0 - cs, 2.0 * (double)gen)) < (1.4 + 2.0 / (kN + 1.0)) * chi_n;
        const double a_c = hs ? std::sqrt(cc * (2.0 - cc) * mueff) : 0.0;
        for (int k = 0; k < kN; ++k) pc[k] = (1.0 - cc) * pc[k] + a_c * yw[k];
        const double keep = 1.0 - c1 - cmu;
        const double hfix = hs ? 0.0 : cc * (2.0 - cc);
        double Cn[kN][kN];
        for (int i = 0; i < kN; ++i)
            for (int j = 0; j < kN; ++j) {
                double r = 0.0;
                for (int t = 0; t < mu; ++t) {
                    const double* yt = &y[(size_t)order[(size_t)t] * kN];
                    r += w[(size_t)t] * yt[i] * yt[j];
                }
                Cn[i][j] = keep * C[i][j] + c1 * (pc[i] * pc[j] + hfix * C[i][j]) + cmu * r;
            }
        for (int i = 0; i < kN; ++i)
            for (int j = 0; j < kN; ++j) C[i][j] = 0.5 * (Cn[i][j] + Cn[j][i]);
        sigma *= std::exp((cs / ds) * (nps / chi_n - 1.0));
    }
};

}  // namespace

extern "C" int rbl_ref_search(const rbl_event* ev, const double* lo, const double* hi, int32_t n_starts,
                              const double* starts, double sigma0, int32_t lambda, int32_t generations,
                              const double* normals, double* best_theta, double* best_lnl, double* trace,
                              int32_t* generations_run, void* hip_stream) {
    if (!ev || !lo || !hi || !starts || !normals || !best_theta || !best_lnl || !generations_run)
        return fail(RBL_EINVAL, "rbl_ref_search: null argument");
    if (!(ev->flags & RBL_KEEP_GRID) || !ev->d_data)
        return fail(RBL_EUNSUPPORTED, "rbl_ref_search: the event was built without RBL_KEEP_GRID");
    if (lambda < 4 || n_starts < 1 || (int64_t)lambda * n_starts > (1 << 20) || generations < 1)
        return fail(RBL_EINVAL, "rbl_ref_search: need lambda >= 4, n_starts >= 1, lambda n_starts <= 2^20 and "
                                "generations >= 1");
    if (!(sigma0 > 0.0) || !std::isfinite(sigma0)) return fail(RBL_EINVAL, "rbl_ref_search: sigma0 must be > 0");
    double width[kN];
    for (int i = 0; i < kN; ++i) {
        if (!(hi[i] > lo[i]) || !std::isfinite(lo[i]) || !std::isfinite(hi[i]))
            return fail(RBL_EINVAL, "rbl_ref_search: the box needs lo < hi, finite");
        width[i] = hi[i] - lo[i];
    }
    const int R = n_starts;
    std::vector<Cmaes> es;
    es.reserve((size_t)R);
    for (int r = 0; r < R; ++r) {
        double u0[kN];
        for (int i = 0; i < kN; ++i) {
            u0[i] = (starts[r * kN + i] - lo[i]) / width[i];
            if (!(u0[i] >= 0.0 && u0[i] <= 1.0)) return fail(RBL_EINVAL, "rbl_ref_search: a start outside the box");
        }
        es.emplace_back(u0, sigma0, lambda);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t L = lambda;
    const int64_t B_max = L * R;
    const int64_t ws_bytes = full_workspace_bytes(ev->n_freq, B_max, ev->waveform);
    DevList mem;
    double *d_theta = nullptr, *d_lnl = nullptr;
    void* d_ws = nullptr;
    if (mem.alloc((void**)&d_theta, sizeof(double) * B_max * kN) != hipSuccess ||
        mem.alloc((void**)&d_lnl, sizeof(double) * B_max) != hipSuccess ||
        mem.alloc(&d_ws, (size_t)ws_bytes) != hipSuccess) {
        mem.release();
        return fail(RBL_ENOMEM, "rbl_ref_search: device allocation");
    }
    std::vector<double> y((size_t)(B_max * kN)), theta((size_t)(B_max * kN)), lnl((size_t)B_max), fit((size_t)L);
    std::vector<char> inside((size_t)B_max), running((size_t)R, 1);
    std::vector<double> run_best((size_t)R, -HUGE_VAL);
    std::vector<int> active;
    double best_f = -HUGE_VAL;
    for (int i = 0; i < kN; ++i) best_theta[i] = starts[i];
    for (int r = 0; r < R; ++r) generations_run[r] = generations;
    int rc = RBL_OK;
    for (int32_t g = 0; g < generations && rc == RBL_OK; ++g) {
        active.clear();
        for (int r = 0; r < R; ++r) {
            if (!running[(size_t)r]) continue;
            if (!es[(size_t)r].factor()) {  // this run has converged as far as its covariance allows
                running[(size_t)r] = 0;
                generations_run[r] = g;
                continue;
            }
            active.push_back(r);
        }
        if (active.empty()) break;
        const int64_t B = L * (int64_t)active.size();
        for (size_t j = 0; j < active.size(); ++j) {
            const Cmaes& e = es[(size_t)active[j]];
            for (int64_t k = 0; k < L; ++k) {
                const int64_t c = (int64_t)j * L + k;
                e.sample(normals + (((int64_t)active[j] * generations + g) * L + k) * kN, &y[(size_t)(c * kN)]);
                bool in = true;
                for (int i = 0; i < kN; ++i) {
                    const double u = e.m[i] + e.sigma * y[(size_t)(c * kN + i)];
                    in = in && u >= 0.0 && u <= 1.0;
                    theta[(size_t)(c * kN + i)] = lo[i] + u * width[i];
                }
                inside[(size_t)c] = in;
            }
        }
        hipError_t e = hipMemcpyAsync(d_theta, theta.data(), sizeof(double) * B * kN, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = launch_chain_setup(d_theta, B, ev->net, ev->ref, (double*)d_ws, nullptr, s);
        if (e == hipSuccess) {
            FullArgs a{};
            a.recs = (const double*)d_ws;
            a.ref = ev->ref;
            a.n_det = ev->n_det;
            a.n_freq = ev->n_freq;
            a.f_low = ev->f_low;
            a.delta_f = ev->delta_f;
            a.data = ev->d_data;
            a.psd = ev->d_psd;
            a.phasor = ev->dev.phasor;
            a.lnl = d_lnl;
            double* consts = (double*)((char*)d_ws + align_up(B * kRecStride * (int64_t)sizeof(double)));
            double* partials = (double*)((char*)consts + align_up(B * kFullStride * (int64_t)sizeof(double)));
            e = launch_loglike_full(a, B, consts, partials, s);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(lnl.data(), d_lnl, sizeof(double) * B, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "rbl_ref_search: fitness evaluation");
            break;
        }
        for (size_t j = 0; j < active.size(); ++j) {
            const int r = active[j];
            int64_t kb = -1;
            for (int64_t k = 0; k < L; ++k) {
                const int64_t c = (int64_t)j * L + k;
                const double f = lnl[(size_t)c];
                fit[(size_t)k] = (inside[(size_t)c] && !std::isnan(f)) ? f : -HUGE_VAL;
                if (kb < 0 || fit[(size_t)k] > fit[(size_t)kb]) kb = k;
            }
            run_best[(size_t)r] = std::max(run_best[(size_t)r], fit[(size_t)kb]);
            if (fit[(size_t)kb] > best_f) {
                best_f = fit[(size_t)kb];
                for (int i = 0; i < kN; ++i) best_theta[i] = theta[(size_t)(((int64_t)j * L + kb) * kN + i)];
            }
            es[(size_t)r].tell(&y[(size_t)((int64_t)j * L * kN)], fit.data());
            if (trace) {
                double* t = trace + ((int64_t)r * generations + g) * (kN + 2);
                t[0] = run_best[(size_t)r];
                t[1] = es[(size_t)r].sigma;
                for (int i = 0; i < kN; ++i) t[2 + i] = lo[i] + es[(size_t)r].m[i] * width[i];
            }
        }
    }
    mem.release();
    *best_lnl = best_f;
    return rc;
}
