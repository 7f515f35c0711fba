// Autotuner of the solver's run-time knobs (not of the method): the sweep
// counts, damping and smoother kind of the multigrid preconditioner of the
// momentum/mass solve, and the sweep count and damping of the band systems'
// preconditioner.  None of them changes the converged answer (FGMRES admits
// any right preconditioner and stops at the same relative residual); the
// definition parameters (band_cell, band_halo, band_flat, eps, eta, dt,
// tolerances) are never touched.
//
// The objective is measured, not modelled: on the caller's state the tuner
// assembles the momentum/mass system once (the first nonlinear iteration of
// a step) and times one full FGMRES solve per candidate, host clock around a
// synchronized solve; then it times one transport pass per band candidate on
// copies of the order parameters and B.  The best candidate is kept in the
// context and, with a cache path, stored under a key of the device
// architecture and the problem's sizes and solver settings, so that a later
// context of the same configuration reads it back instead of searching.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "eft_internal.h"

namespace {

__global__ void k_apply_dir(int64_t n_dir, const int32_t *node, const uint8_t *mask, const double *val, int BS,
                            double *vp)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_dir) return;
    const int64_t n = node[t];
    for (int i = 0; i < BS; ++i)
        if ((mask[t] >> i) & 1) vp[n * BS + i] = val[t * BS + i];
}

__global__ void k_negate_copy(const double *a, double *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = -a[i];
}

struct Knobs {
    int mg_nu, mg_nu_post, mg_smoother;
    double mg_omega;
    int mg_galerkin;
    int band_sweeps;
    double band_omega;
    int mg_cnu, mg_cnu_post;
};

Knobs knobs_of(const eft_params &p)
{
    return Knobs{p.mg_nu,       p.mg_nu_post, p.mg_smoother, p.mg_omega,   p.mg_galerkin,
                 p.band_sweeps, p.band_omega, p.mg_cnu,      p.mg_cnu_post};
}

void set_knobs(eft_params &p, const Knobs &k)
{
    p.mg_nu = k.mg_nu;
    p.mg_nu_post = k.mg_nu_post;
    p.mg_smoother = k.mg_smoother;
    p.mg_omega = k.mg_omega;
    p.mg_galerkin = k.mg_galerkin;
    p.band_sweeps = k.band_sweeps;
    p.band_omega = k.band_omega;
    p.mg_cnu = k.mg_cnu;
    p.mg_cnu_post = k.mg_cnu_post;
}

std::string knobs_text(const Knobs &k)
{
    char b[256];
    std::snprintf(b, sizeof b,
                  "mg_nu=%d mg_nu_post=%d mg_smoother=%d mg_omega=%.6g mg_galerkin=%d band_sweeps=%d band_omega=%.6g "
                  "mg_cnu=%d mg_cnu_post=%d",
                  k.mg_nu, k.mg_nu_post, k.mg_smoother, k.mg_omega, k.mg_galerkin, k.band_sweeps, k.band_omega,
                  k.mg_cnu, k.mg_cnu_post);
    return b;
}

bool parse_knobs(const std::string &s, Knobs &k)
{
    return std::sscanf(s.c_str(),
                       "mg_nu=%d mg_nu_post=%d mg_smoother=%d mg_omega=%lf mg_galerkin=%d band_sweeps=%d band_omega=%lf "
                       "mg_cnu=%d mg_cnu_post=%d",
                       &k.mg_nu, &k.mg_nu_post, &k.mg_smoother, &k.mg_omega, &k.mg_galerkin, &k.band_sweeps,
                       &k.band_omega, &k.mg_cnu, &k.mg_cnu_post) == 9;
}

std::string tune_key(eft_ctx *ctx)
{
    int dev = 0;
    std::string arch = "unknown";
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char &c : arch)
        if (c == ' ' || c == '|') c = '_';
    const eft_params &p = ctx->par;
    std::ostringstream o;
    o << arch << " d" << ctx->dim << " N" << ctx->N << " E" << ctx->E << " nnzb" << ctx->J.nnzb << " ind" << ctx->n_ind
      << " s" << ctx->n_s << " prec" << p.precision << " pc" << p.precond << " m" << p.restart << " bf16" << p.mg_bf16
      << " rtol" << p.lin_rtol << " dt" << p.dt;
    for (int ph = 0; ph < ctx->n_phase; ++ph)
        o << " ph" << ctx->phase[ph].rho << "/" << ctx->phase[ph].mu << "/" << ctx->phase[ph].mu_L;
    return o.str();
}

bool cache_lookup(const char *path, const std::string &key, Knobs &k)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {   // the last entry of a key wins
        const size_t bar = line.find('|');
        if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
        Knobs t;
        if (parse_knobs(line.substr(bar + 1), t)) {
            k = t;
            found = true;
        }
    }
    return found;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" eft_status eft_tune(eft_ctx *ctx, const eft_state *st, const char *cache_path, int32_t budget,
                               eft_tune_info *info)
{
    if (!ctx || !st || !st->vp || !st->vdot) return EFT_EINVAL;
    if ((ctx->n_ind > 0 && (!st->phi || !st->phidot)) || (ctx->n_s > 0 && (!st->B || !st->Bdot))) return EFT_EINVAL;
    eft_tune_info inf{};
    const Knobs entry = knobs_of(ctx->par);
    const std::string key = tune_key(ctx);
    Knobs best = entry;
    if (cache_lookup(cache_path, key, best)) {
        set_knobs(ctx->par, best);
        EFT_TRY(eft_set_params(ctx, &ctx->par));
        inf.from_cache = 1;
        inf.mg_nu = best.mg_nu;
        inf.mg_nu_post = best.mg_nu_post;
        inf.mg_smoother = best.mg_smoother;
        inf.mg_omega = best.mg_omega;
        inf.mg_galerkin = best.mg_galerkin;
        inf.mg_cnu = best.mg_cnu;
        inf.mg_cnu_post = best.mg_cnu_post;
        inf.band_sweeps = best.band_sweeps;
        inf.band_omega = best.band_omega;
        if (info) *info = inf;
        return EFT_OK;
    }
    const int cap = budget > 0 ? budget : 96;
    const int64_t N = ctx->N;
    const int bs = ctx->bs, nv = ctx->nv;
    const int64_t nvp = N * bs, nphi = N * ctx->n_ind, nB = N * nv * ctx->n_s;
    // the first iterate of a step: level values, predictor with boundary data
    double *it_vp = nullptr, *it_phi = nullptr, *it_B = nullptr, *b = nullptr, *x = nullptr;
    auto release = [&]() {
        for (double *p : {it_vp, it_phi, it_B, b, x})
            if (p) (void)hipFree(p);
    };
    if (hipMalloc(&it_vp, sizeof(double) * nvp) != hipSuccess || hipMalloc(&b, sizeof(double) * nvp) != hipSuccess ||
        hipMalloc(&x, sizeof(double) * nvp) != hipSuccess ||
        (nphi && hipMalloc(&it_phi, sizeof(double) * nphi) != hipSuccess) ||
        (nB && hipMalloc(&it_B, sizeof(double) * nB) != hipSuccess)) {
        release();
        ctx->err = "out of device memory (tuner)";
        return EFT_ENOMEM;
    }
    eft_status stt = EFT_OK;
    auto fail = [&](eft_status s) {
        release();
        set_knobs(ctx->par, entry);
        return s;
    };
#define TUNE_TRY(expr)                       \
    do {                                     \
        eft_status s_ = (expr);              \
        if (s_ != EFT_OK) return fail(s_);   \
    } while (0)
    TUNE_TRY(hipMemcpyAsync(it_vp, st->vp, sizeof(double) * nvp, hipMemcpyDeviceToDevice, ctx->stream) == hipSuccess
                 ? EFT_OK
                 : EFT_EDEVICE);
    if (ctx->n_dir > 0)
        hipLaunchKernelGGL(k_apply_dir, dim3(eft_grid(ctx->n_dir, 128)), dim3(128), 0, ctx->stream, ctx->n_dir,
                           ctx->dir_node, ctx->dir_mask, ctx->dir_val, bs, it_vp);
    eft_iterate it{it_vp, nphi ? st->phi : nullptr, nB ? st->B : nullptr};
    TUNE_TRY(eft_props(ctx, st, &it));
    TUNE_TRY(eft_ns_kernels(ctx, &it, ctx->R, &ctx->J));
    hipLaunchKernelGGL(k_negate_copy, dim3(eft_grid(nvp, 256)), dim3(256), 0, ctx->stream, ctx->R, b, nvp);
    TUNE_TRY(hipStreamSynchronize(ctx->stream) == hipSuccess ? EFT_OK : EFT_EDEVICE);
    const int maxit0 = ctx->par.lin_maxit;
    // the entry settings may be poor (or stall): their solves stop at a
    // bounded count too, and a solve that does not converge there is no
    // candidate
    const int cap_entry = std::min(maxit0, 400);
    int evaluated = 0;
    // one timed momentum solve with the knobs k (iterations capped so that a
    // poor candidate cannot run for long); seconds, or a negative value when
    // it did not converge
    auto time_solve = [&](const Knobs &k, int cap_it, int *iters) -> double {
        set_knobs(ctx->par, k);
        ctx->par.lin_maxit = std::max(1, std::min(maxit0, cap_it));
        eft_solve_info si{};
        (void)hipStreamSynchronize(ctx->stream);
        const double t0 = now_s();
        stt = eft_fgmres_dev(ctx, &ctx->J, b, x, &si);
        (void)hipStreamSynchronize(ctx->stream);
        const double t = now_s() - t0;
        ctx->par.lin_maxit = maxit0;
        ++evaluated;
        *iters = si.iters;
        if (stt == EFT_ENOTCONV) {
            stt = EFT_OK;
            return -1.0;
        }
        return si.converged ? t : -1.0;
    };
    // ---- momentum/mass: multigrid knobs (only with the multigrid active)
    double t_entry = 0.0, t_best = 0.0;
    int it_entry = 0, it_best = 0;
    if (eft_mg_active(ctx, &ctx->J)) {
        int itw = 0;
        (void)time_solve(entry, cap_entry, &itw);   // warm-up (first use of the kernels)
        if (stt != EFT_OK) return fail(stt);
        t_entry = time_solve(entry, cap_entry, &it_entry);
        if (stt != EFT_OK) return fail(stt);
        t_best = t_entry > 0.0 ? t_entry : 1e300;
        it_best = t_entry > 0.0 ? it_entry : 100;
        auto consider = [&](Knobs k) -> eft_status {
            if (evaluated >= cap) return EFT_OK;
            int its = 0;
            const double t = time_solve(k, std::max(8, 3 * std::max(it_best, 1)), &its);
            if (stt != EFT_OK) return stt;
            if (t > 0.0 && t < t_best) {
                t_best = t;
                it_best = its;
                best = k;
            }
            return EFT_OK;
        };
        // (pre, post) sweep pairs of the grid, each at two dampings: the best
        // pairs move with the damping, so neither is fixed first
        const int pairs[][2] = {{1, 2}, {1, 3}, {1, 4}, {2, 2}, {2, 3}, {2, 4}, {3, 3}, {3, 4},
                                {4, 4}, {4, 6}, {4, 8}, {6, 6}, {8, 8}, {2, 8}, {1, 8}};
        const double omegas[] = {0.75, 0.85};
        // both kinds of coarse operators; switching rebuilds the hierarchy
        // (the assembly's set-up of the multigrid levels) before the timings
        const int gal0 = entry.mg_galerkin;
        for (int gi = 0; gi < 2; ++gi) {
            const int gal = gi == 0 ? gal0 : 1 - gal0;
            if (gal != ctx->par.mg_galerkin) {
                ctx->par.mg_galerkin = gal;
                TUNE_TRY(eft_ns_kernels(ctx, &it, ctx->R, &ctx->J));
                TUNE_TRY(hipStreamSynchronize(ctx->stream) == hipSuccess ? EFT_OK : EFT_EDEVICE);
            }
            for (double om : omegas)
                for (const auto &pc : pairs) {
                    Knobs k = best;
                    k.mg_galerkin = gal;
                    k.mg_smoother = 0;
                    k.mg_omega = om;
                    k.mg_nu = pc[0];
                    k.mg_nu_post = pc[1];
                    TUNE_TRY(consider(k));
                }
        }
        // the hierarchy of the best candidate's coarse operators
        if (best.mg_galerkin != ctx->par.mg_galerkin) {
            ctx->par.mg_galerkin = best.mg_galerkin;
            TUNE_TRY(eft_ns_kernels(ctx, &it, ctx->R, &ctx->J));
        }
        for (double om : {0.65, 0.95}) {
            Knobs k = best;
            k.mg_omega = om;
            TUNE_TRY(consider(k));
        }
        {   // the multicolour Gauss-Seidel smoother at the same and at half the sweeps
            Knobs k = best;
            k.mg_smoother = 1;
            TUNE_TRY(consider(k));
            k.mg_nu = std::max(1, best.mg_nu / 2);
            k.mg_nu_post = std::max(1, best.mg_nu_post / 2);
            TUNE_TRY(consider(k));
        }
        // the coarse levels' own sweep counts at the best finest counts (the
        // coarse correction sets the convergence of the cycle, and a coarse
        // sweep costs an eighth of a finest one), then the finest counts
        // again at the best coarse ones
        for (int c : {4, 6, 8, 12}) {
            Knobs k = best;
            k.mg_cnu = c;
            k.mg_cnu_post = c;
            TUNE_TRY(consider(k));
        }
        if (best.mg_cnu > 0) {
            const int fine[][2] = {{1, 1}, {1, 2}, {2, 2}, {2, 3}, {2, 4}, {3, 3}};
            for (const auto &f : fine) {
                Knobs k = best;
                if (k.mg_nu == f[0] && k.mg_nu_post == f[1]) continue;
                k.mg_nu = f[0];
                k.mg_nu_post = f[1];
                TUNE_TRY(consider(k));
            }
        }
        // confirm against the entry settings with a second timing of both
        if (!(best.mg_nu == entry.mg_nu && best.mg_nu_post == entry.mg_nu_post &&
              best.mg_smoother == entry.mg_smoother && best.mg_omega == entry.mg_omega &&
              best.mg_galerkin == entry.mg_galerkin && best.mg_cnu == entry.mg_cnu &&
              best.mg_cnu_post == entry.mg_cnu_post)) {
            int i1 = 0, i2 = 0;
            const double t1 = time_solve(best, cap_entry, &i1);
            double t2 = t_entry;
            if (entry.mg_galerkin == best.mg_galerkin) t2 = time_solve(entry, cap_entry, &i2);
            else i2 = it_entry;
            if (stt != EFT_OK) return fail(stt);
            if (!(t1 > 0.0) || (t2 > 0.0 && t2 <= t1)) {
                if (best.mg_galerkin != entry.mg_galerkin) {
                    ctx->par.mg_galerkin = entry.mg_galerkin;
                    TUNE_TRY(eft_ns_kernels(ctx, &it, ctx->R, &ctx->J));
                }
                best.mg_nu = entry.mg_nu;
                best.mg_nu_post = entry.mg_nu_post;
                best.mg_smoother = entry.mg_smoother;
                best.mg_omega = entry.mg_omega;
                best.mg_galerkin = entry.mg_galerkin;
                best.mg_cnu = entry.mg_cnu;
                best.mg_cnu_post = entry.mg_cnu_post;
                t_best = t2;
                it_best = i2;
            } else {
                t_best = t1;
                it_best = i1;
            }
        }
    }
    inf.default_seconds = t_entry;
    inf.best_seconds = t_best;
    inf.default_iters = it_entry;
    inf.best_iters = it_best;
    set_knobs(ctx->par, best);
    // ---- band systems: sweeps and damping of their preconditioner
    if (ctx->n_ind > 0) {
        TUNE_TRY(eft_bands_build_dev(ctx, st->phi));
        auto time_transport = [&](const Knobs &k) -> double {
            set_knobs(ctx->par, k);
            if (nphi) (void)hipMemcpyAsync(it_phi, st->phi, sizeof(double) * nphi, hipMemcpyDeviceToDevice, ctx->stream);
            if (nB) (void)hipMemcpyAsync(it_B, st->B, sizeof(double) * nB, hipMemcpyDeviceToDevice, ctx->stream);
            eft_iterate tit{it_vp, it_phi, it_B};
            eft_transport_info ti{};
            (void)hipStreamSynchronize(ctx->stream);
            const double t0 = now_s();
            stt = eft_transport_dev(ctx, st, &tit, &ti);
            (void)hipStreamSynchronize(ctx->stream);
            ++evaluated;
            if (stt == EFT_ENOTCONV) {
                stt = EFT_OK;
                return -1.0;
            }
            return now_s() - t0;
        };
        (void)time_transport(best);   // warm-up
        if (stt != EFT_OK) return fail(stt);
        const double tb0 = time_transport(best);
        if (stt != EFT_OK) return fail(stt);
        double tbb = tb0 > 0.0 ? tb0 : 1e300;
        Knobs bb = best;
        for (int sw : {1, 2, 3, 4})
            for (double om : {0.5, 0.6, 0.7}) {
                if (evaluated >= cap + 16) break;
                Knobs k = best;
                k.band_sweeps = sw;
                k.band_omega = om;
                if (sw == best.band_sweeps && om == best.band_omega) continue;
                const double t = time_transport(k);
                if (stt != EFT_OK) return fail(stt);
                if (t > 0.0 && t < tbb) {
                    tbb = t;
                    bb = k;
                }
            }
        inf.band_default_seconds = tb0;
        inf.band_best_seconds = tbb < 1e300 ? tbb : tb0;
        best = bb;
        ctx->bands_valid = false;
    }
#undef TUNE_TRY
    release();
    set_knobs(ctx->par, best);
    EFT_TRY(eft_set_params(ctx, &ctx->par));
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f) f << key << "|" << knobs_text(best) << "\n";
    }
    inf.evaluated = evaluated;
    inf.mg_nu = best.mg_nu;
    inf.mg_nu_post = best.mg_nu_post;
    inf.mg_smoother = best.mg_smoother;
    inf.mg_omega = best.mg_omega;
    inf.mg_galerkin = best.mg_galerkin;
    inf.mg_cnu = best.mg_cnu;
    inf.mg_cnu_post = best.mg_cnu_post;
    inf.band_sweeps = best.band_sweeps;
    inf.band_omega = best.band_omega;
    if (info) *info = inf;
    return EFT_OK;
}
