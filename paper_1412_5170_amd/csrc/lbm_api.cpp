// C ABI runtime of the pseudo-potential D2Q9 lattice Boltzmann library (include/pplbm.h):
// parameter validation, Carnahan-Starling critical point and Maxwell densities on the host,
// device buffers, the time-step launch sequence and the read-back paths.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pplbm.h"
#include "lbm_internal.h"

using pplbm::Physics;

struct lbm {
    Physics p{};
    lbm_eos eos{};
    lbm_force force{};
    lbm_collision coll{};
    double tau = 1.0, T = 0.0;
    float *f[2] = {nullptr, nullptr};
    float *psi = nullptr;
    bool owned = false;
    int cur = 0;  // index of the buffer holding the current populations
    hipStream_t stream = nullptr;
    int prec = pplbm::kPrecMixed;  // arithmetic precision (see lbm_set_precision)
    int layout = LBM_LAYOUT_ROWS;
    pplbm::Launch launch;
    int xa = 0, ya = 0, xb = 0, yb = 0;
    long long step = 0;
    bool initialised = false;
    float *vprev = nullptr;
    bool vprev_valid = false;
    double *stats_partial = nullptr;
    double *stats_out = nullptr;
    bool timing = false;
    std::vector<hipEvent_t> events;  // 3 per timed step not yet folded into the sums
    size_t events_used = 0;
    long long timed_steps = 0;
    double timed_a = 0.0, timed_b = 0.0;  // folded milliseconds (psi pass, main pass)
    std::string err;
};

namespace {

int fail(lbm *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(lbm *h, hipError_t e, const char *what) {
    if (h) h->err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EHIP;
}

#define HIP_TRY(h, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

// ---- Carnahan-Starling EOS on the host (Eq. 29-30), written in eta = b rho / 4 ----------
// p(eta) = K [ (4 R T / b) h(eta) - (16 a / b^2) eta^2 ],  h = eta Z(eta),
// Z = (1 + eta + eta^2 - eta^3) / (1 - eta)^3.
struct CS {
    double a, b, R, K;
    double dpdrho(double rho, double T) const {
        // d(rho Z)/drho = Z + eta Z',  Z' = (4 + 4 eta - 2 eta^2) / (1 - eta)^4
        const double eta = b * rho / 4.0, om = 1.0 - eta;
        const double Z = (1.0 + eta + eta * eta - eta * eta * eta) / (om * om * om);
        const double dZ = (4.0 + 4.0 * eta - 2.0 * eta * eta) / (om * om * om * om);
        return K * (R * T * (Z + eta * dZ) - 2.0 * a * rho);
    }
    double p(double rho, double T) const {
        const double eta = b * rho / 4.0, om = 1.0 - eta;
        const double Z = (1.0 + eta + eta * eta - eta * eta * eta) / (om * om * om);
        return K * (rho * R * T * Z - a * rho * rho);
    }
    // Gibbs energy per particle up to a constant, from the Helmholtz energy per particle
    // R T (ln rho - 1 + (4 eta - 3 eta^2)/(1 - eta)^2) - a rho (whose rho^2 d/drho is p / K).
    double g(double rho, double T) const {
        const double eta = b * rho / 4.0, om = 1.0 - eta;
        const double f = R * T * (std::log(rho) - 1.0 + (4.0 * eta - 3.0 * eta * eta) / (om * om)) - a * rho;
        return K * f + p(rho, T) / rho;
    }
};

// Critical point: with h(eta) = N / (1 - eta)^3, N = eta + eta^2 + eta^3 - eta^4,
// dp/deta = 0 and d2p/deta2 = 0 give h'(eta) = eta h''(eta) (independent of a, b, R) and
// T_c = 8 a / (b R h''(eta_c)).
void critical(double a, double b, double R, double *rho_c, double *T_c, double *p_c) {
    auto h1 = [](double e) {
        const double N = e + e * e + e * e * e - e * e * e * e, N1 = 1 + 2 * e + 3 * e * e - 4 * e * e * e;
        const double D = 1 - e;
        return N1 / (D * D * D) + 3 * N / (D * D * D * D);
    };
    auto h2 = [](double e) {
        const double N = e + e * e + e * e * e - e * e * e * e, N1 = 1 + 2 * e + 3 * e * e - 4 * e * e * e;
        const double N2 = 2 + 6 * e - 12 * e * e, D = 1 - e;
        return N2 / (D * D * D) + 6 * N1 / (D * D * D * D) + 12 * N / (D * D * D * D * D);
    };
    double lo = 0.05, hi = 0.3;  // g(lo) > 0 > g(hi) for g = h' - eta h''
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (h1(mid) - mid * h2(mid) > 0) lo = mid; else hi = mid;
    }
    const double ec = 0.5 * (lo + hi);
    const double Tc = 8.0 * a / (b * R * h2(ec));
    const double rc = 4.0 * ec / b;
    CS cs{a, b, R, 1.0};
    if (rho_c) *rho_c = rc;
    if (T_c) *T_c = Tc;
    if (p_c) *p_c = cs.p(rc, Tc);
}

// Root of an increasing function on [lo, hi] by bisection to the last bit.
template <typename F>
double bisect_up(F fn, double lo, double hi) {
    for (int it = 0; it < 300; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (fn(mid) < 0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

int maxwell(const lbm_eos &e, double *rho_g, double *rho_l) {
    double rc, Tc, pc;
    critical(e.a, e.b, e.R, &rc, &Tc, &pc);
    const double T = e.T_over_Tc * Tc;
    const CS cs{e.a, e.b, e.R, 1.0};  // the densities do not depend on K
    const double rmax = 4.0 / e.b;
    auto dp = [&](double r) { return cs.dpdrho(r, T); };
    // Spinodals: local maximum below rho_c and local minimum above it.
    const double s1 = bisect_up([&](double r) { return -dp(r); }, 1e-9 * rmax, rc);
    const double s2 = bisect_up(dp, rc, 0.999 * rmax);
    if (!(s1 < s2) || !(dp(0.5 * (s1 + s2)) < 0)) return LBM_EINVAL;
    const double plo = std::fmax(cs.p(s2, T), 0.0), phi = cs.p(s1, T);
    auto branches = [&](double P, double *g, double *l) {
        *g = bisect_up([&](double r) { return cs.p(r, T) - P; }, 1e-300, s1);
        double hi = s2 + 0.5 * (rmax - s2);
        while (cs.p(hi, T) < P) hi = rmax - 0.5 * (rmax - hi);
        *l = bisect_up([&](double r) { return cs.p(r, T) - P; }, s2, hi);
    };
    // Equal chemical potential: g(rho_g) - g(rho_l) rises with the trial pressure (at the low
    // end rho_g -> 0 and its ln rho_g -> -inf).
    double g = 0, l = 0;
    const double P = bisect_up([&](double P) {
        double gg, ll;
        branches(P, &gg, &ll);
        return cs.g(gg, T) - cs.g(ll, T);
    }, plo + 1e-15 * phi, phi * (1 - 1e-12));
    branches(P, &g, &l);
    *rho_g = g;
    *rho_l = l;
    return LBM_OK;
}

// Shape of the one-step sweep, which also runs the odd last step of a two-step lbm_step call:
// strips as wide as 512 columns and segments as tall as 8 rows, two rows of loads in flight
// and XCD-ordered tiles (its fastest measured shape on MRT droplets from 2048^2 to 8192^2),
// narrowed and shortened (down to 64 x 4) until the launch has about 1024 workgroups to spread
// over the 256 compute units.
pplbm::Launch default_launch(int nx, int ny) {
    pplbm::Launch L;
    L.kernel = pplbm::kKernelSweep;
    L.flags = pplbm::kFlagXCD;
    L.tx = 512;
    L.ty = 8;
    auto groups = [&]() {
        return (double)(((long long)nx + L.tx - 1) / L.tx) * (((long long)ny + L.ty - 1) / L.ty);
    };
    while (groups() < 1024 && (L.tx > 64 || L.ty > 4)) {
        if (L.tx > 64 && (L.tx >= 2 * 64 && nx <= L.tx * 4)) L.tx /= 2;
        else if (L.ty > 4) L.ty /= 2;
        else L.tx /= 2;
    }
    return L;
}

int validate(int nx, int ny, const lbm_eos *eos, const lbm_force *force,
             const lbm_collision *coll, double tau, std::string *why) {
    auto bad = [&](const char *m) { *why = m; return LBM_EINVAL; };
    if (!eos || !force || !coll) return bad("null parameter struct");
    if (nx < 1 || ny < 1) return bad("nx and ny must be >= 1");
    if ((double)nx * (double)ny > 4.0e9) return bad("lattice too large");
    if (!(tau > 0.5) || !std::isfinite(tau)) return bad("tau must be > 1/2");
    if (eos->kind == LBM_EOS_CARNAHAN_STARLING) {
        if (!(eos->a > 0) || !(eos->b > 0) || !(eos->R > 0) || !(eos->K > 0))
            return bad("EOS constants a, b, R, K must be positive");
        if (!(eos->T_over_Tc > 0) || !std::isfinite(eos->T_over_Tc)) return bad("T/Tc must be positive");
    } else if (eos->kind == LBM_EOS_SBRAGAGLIA_SHAN) {
        if (!(eos->eps >= 0) || !std::isfinite(eos->eps)) return bad("Eq. 33 exponent eps must be >= 0");
    } else {
        return bad("unknown EOS kind");
    }
    if (!(force->G < 0)) return bad("G must be negative (Eq. 7 needs 2 U / G > 0)");
    if (force->scheme < LBM_FORCE_EDM || force->scheme > LBM_FORCE_SC) return bad("unknown forcing scheme");
    if (!std::isfinite(force->A) || !std::isfinite(force->sigma)) return bad("A and sigma must be finite");
    if (coll->kind != LBM_COLL_BGK && coll->kind != LBM_COLL_MRT) return bad("unknown collision");
    if (coll->kind == LBM_COLL_MRT) {
        if (force->scheme == LBM_FORCE_EDM || force->scheme == LBM_FORCE_SC)
            return bad("MRT is defined with Guo's forcing only");
        const double r[5] = {coll->s_rho, coll->s_e, coll->s_eps, coll->s_j, coll->s_q};
        for (double s : r)
            if (!(s > 0 && s < 2)) return bad("MRT rates must lie in (0, 2)");
    }
    return LBM_OK;
}

// The sweep addresses populations with 32-bit buffer offsets: the whole buffer below 4 GiB,
// else one resource per row, which needs the row-interleaved layout (a row's nine planes
// within 9 x pitch floats).
bool sweep_fits(const lbm *h) {
    return pplbm::pop_bytes(h->p) <= pplbm::kSweepMaxBytes || h->layout == LBM_LAYOUT_ROWS;
}

int ensure_buffers(lbm *h) {
    if (h->f[0]) return LBM_OK;
    size_t fb, pb;
    lbm_layout(h, nullptr, nullptr, &fb, &pb);
    void *a = nullptr, *b = nullptr, *c = nullptr;
    if (hipMalloc(&a, fb) != hipSuccess || hipMalloc(&b, fb) != hipSuccess ||
        hipMalloc(&c, pb) != hipSuccess) {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (c) (void)hipFree(c);
        (void)hipGetLastError();
        return fail(h, LBM_ENOMEM, "device allocation of the lattice buffers failed");
    }
    h->f[0] = (float *)a;
    h->f[1] = (float *)b;
    h->psi = (float *)c;
    h->owned = true;
    // Padding columns are never read; clear them once so copies of the planes are defined.
    HIP_TRY(h, hipMemsetAsync(a, 0, fb, h->stream));
    HIP_TRY(h, hipMemsetAsync(b, 0, fb, h->stream));
    HIP_TRY(h, hipMemsetAsync(c, 0, pb, h->stream));
    return LBM_OK;
}

void release_buffers(lbm *h) {
    if (h->owned) {
        (void)hipFree(h->f[0]);
        (void)hipFree(h->f[1]);
        (void)hipFree(h->psi);
    }
    h->f[0] = h->f[1] = h->psi = nullptr;
    h->owned = false;
}

int ensure_stats(lbm *h) {
    if (h->stats_partial && h->stats_out) return LBM_OK;
    const size_t n = pplbm::stats_partial_count(h->p) * pplbm::kStatsFields;
    double *part = nullptr, *out = nullptr;
    if (hipMalloc(&part, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&out, pplbm::kStatsOut * sizeof(double)) != hipSuccess) {
        if (part) (void)hipFree(part);
        (void)hipGetLastError();
        return fail(h, LBM_ENOMEM, "device allocation of the reduction buffers failed");
    }
    h->stats_partial = part;
    h->stats_out = out;
    return LBM_OK;
}

// Timing events are folded into running sums once this many triples are pending, so a long
// timed run holds a bounded number of events (one host synchronisation per fold).
constexpr size_t kTimingFoldSteps = 1024;

int fold_timing(lbm *h) {
    if (h->events_used == 0) return LBM_OK;
    HIP_TRY(h, hipEventSynchronize(h->events[h->events_used - 1]));
    for (size_t k = 0; k + 3 <= h->events_used; k += 3) {
        float t1 = 0, t2 = 0;
        HIP_TRY(h, hipEventElapsedTime(&t1, h->events[k], h->events[k + 1]));
        HIP_TRY(h, hipEventElapsedTime(&t2, h->events[k + 1], h->events[k + 2]));
        h->timed_a += t1;
        h->timed_b += t2;
    }
    h->events_used = 0;
    return LBM_OK;
}

}  // namespace

namespace pplbm {

void critical_point(double a, double b, double R, double *rho_c, double *T_c, double *p_c) {
    critical(a, b, R, rho_c, T_c, p_c);
}

int make_physics(int nx, int ny, const lbm_eos *eos, const lbm_force *force,
                 const lbm_collision *collision, double tau, Physics *out, double *T_out,
                 std::string *why) {
    int rc = validate(nx, ny, eos, force, collision, tau, why);
    if (rc) return rc;
    double T = 0.0;
    if (eos->kind == LBM_EOS_CARNAHAN_STARLING) {
        double rc_, Tc, pc;
        critical(eos->a, eos->b, eos->R, &rc_, &Tc, &pc);
        T = eos->T_over_Tc * Tc;
    }
    Physics p{};
    p.nx = nx;
    p.ny = ny;
    p.pitch = ((size_t)nx + 63) / 64 * 64;
    p.plane = p.pitch * (size_t)ny;
    p.frow = 9 * p.pitch;  // LBM_LAYOUT_ROWS
    p.fq = p.pitch;
    p.b_quarter = eos->b / 4.0;
    p.RT = eos->R * T;
    p.a = eos->a;
    p.K = eos->K;
    p.G = force->G;
    p.A = force->A;
    p.sigma = force->scheme == LBM_FORCE_GUO_LI ? force->sigma : 0.0;
    p.tau = tau;
    p.psi_kind = eos->kind == LBM_EOS_SBRAGAGLIA_SHAN ? 1 : 0;
    p.inv_eps = (p.psi_kind == 1 && eos->eps > 0) ? 1.0 / eos->eps : 0.0;
    p.scheme = force->scheme;
    p.coll = collision->kind;
    const double snu = 1.0 / tau;
    if (collision->kind == LBM_COLL_MRT) {
        const double s[9] = {collision->s_rho, collision->s_e, collision->s_eps, collision->s_j,
                             collision->s_q, collision->s_j, collision->s_q, snu, snu};
        std::memcpy(p.s, s, sizeof s);
    } else {
        for (double &s : p.s) s = snu;
    }
    *out = p;
    if (T_out) *T_out = T;
    return LBM_OK;
}

}  // namespace pplbm

extern "C" {

int lbm_create(int nx, int ny, const lbm_eos *eos, const lbm_force *force,
               const lbm_collision *collision, double tau, lbm_t **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    Physics p;
    double T;
    std::string why;
    int rc = pplbm::make_physics(nx, ny, eos, force, collision, tau, &p, &T, &why);
    if (rc) return rc;
    lbm *h = new (std::nothrow) lbm();
    if (!h) return LBM_ENOMEM;
    h->eos = *eos;
    h->force = *force;
    h->coll = *collision;
    h->tau = tau;
    h->T = T;
    h->p = p;
    h->xa = nx / 2;
    h->ya = ny / 2;
    // Two steps per launch (256 threads, four waves of 58 output columns), with per-row
    // resources beyond 4 GiB of populations.  Segment heights, measured on square MRT droplets:
    // 16 rows where that makes at least 8192 waves (shorter waves balance better: +1 % at
    // 4096^2, +3 % at 3000^2 and 6000^2, +4 % at 8192^2 over 24 rows); else 24 rows where that
    // still makes about 3072 waves (2048^2: 16 rows would leave a short second round, 7 %
    // slower); on smaller lattices the height that gives about 3200 waves, one resident round,
    // but at least 6 rows, below which the recomputed rows of step t cost more than the extra
    // waves gain (512^2: +14 %, 768^2: +21 %, 1024^2: +13 %, 1536^2: +7 % over the one-step
    // sweep) -- except where 6 rows leave the GPU partly idle (lattices up to about 1024^2):
    // there the busiest SIMD sets the time, and two_step_height picks 1-12 rows by its waves per
    // SIMD and rows per wave, one wave per workgroup (us per step against 6 rows: 4 x 256 slab
    // 3.85 vs 9.02, 128^2 3.81 vs 7.16, 256^2 4.62 vs 7.35, 384^2 5.51 vs 7.47, 512^2 7.09 vs
    // 7.73, 640^2 8.60 vs 10.43, 832^2 11.81 vs 13.56, 1024^2 14.80 vs 15.51; 768^2 keeps 6).
    // The one-step sweep's default shape serves the odd last step.
    h->launch = default_launch(nx, ny);
    {
        const long long strips = ((long long)nx + 57) / 58;
        bool small = false;
        h->launch.kernel = pplbm::kKernelSweep2;
        h->launch.ty = pplbm::two_step_height(
            [&](int rows) { return strips * (((long long)ny + rows - 1) / rows); }, &small);
        h->launch.tx = small ? 64 : 256;
        h->launch.flags = pplbm::kFlagXCD;  // 4096^2: 167.8 -> 159.2 us per step
    }
    *out = h;
    return LBM_OK;
}

void lbm_destroy(lbm_t *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    release_buffers(h);
    if (h->vprev) (void)hipFree(h->vprev);
    if (h->stats_partial) (void)hipFree(h->stats_partial);
    if (h->stats_out) (void)hipFree(h->stats_out);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    delete h;
}

int lbm_layout(const lbm_t *h, size_t *pitch_floats, size_t *plane_floats, size_t *f_bytes,
               size_t *psi_bytes) {
    if (!h) return LBM_EINVAL;
    if (pitch_floats) *pitch_floats = h->p.pitch;
    if (plane_floats) *plane_floats = h->p.plane;
    if (f_bytes) *f_bytes = 9 * h->p.plane * sizeof(float);
    if (psi_bytes) *psi_bytes = h->p.plane * sizeof(float);
    return LBM_OK;
}

int lbm_attach(lbm_t *h, void *f_a, void *f_b, void *psi, void *stream) {
    if (!h) return LBM_EINVAL;
    if (!f_a || !f_b || !psi || f_a == f_b) return fail(h, LBM_EINVAL, "attach needs three distinct buffers");
    if (((uintptr_t)f_a | (uintptr_t)f_b | (uintptr_t)psi) & 255)
        return fail(h, LBM_EINVAL, "attached buffers must be 256-byte aligned");
    release_buffers(h);
    h->f[0] = (float *)f_a;
    h->f[1] = (float *)f_b;
    h->psi = (float *)psi;
    h->owned = false;
    h->stream = (hipStream_t)stream;
    h->cur = 0;
    h->initialised = false;
    return LBM_OK;
}

int lbm_set_stream(lbm_t *h, void *stream) {
    if (!h) return LBM_EINVAL;
    h->stream = (hipStream_t)stream;
    return LBM_OK;
}

int lbm_set_precision(lbm_t *h, int precision) {
    if (!h) return LBM_EINVAL;
    if (precision != LBM_PREC_F64 && precision != LBM_PREC_MIXED)
        return fail(h, LBM_EINVAL, "precision must be LBM_PREC_MIXED or LBM_PREC_F64 (FP32 "
                                   "arithmetic throughout misses 1e-5 after 100 steps and is not offered)");
    h->prec = precision;
    return LBM_OK;
}

int lbm_set_layout(lbm_t *h, int layout) {
    if (!h) return LBM_EINVAL;
    if (layout != LBM_LAYOUT_PLANES && layout != LBM_LAYOUT_ROWS)
        return fail(h, LBM_EINVAL, "layout must be LBM_LAYOUT_PLANES or LBM_LAYOUT_ROWS");
    if (h->initialised) return fail(h, LBM_ESTATE, "the layout is fixed once the lattice is initialised");
    h->layout = layout;
    h->p.frow = layout == LBM_LAYOUT_ROWS ? 9 * h->p.pitch : h->p.pitch;
    h->p.fq = layout == LBM_LAYOUT_ROWS ? h->p.pitch : h->p.plane;
    if (!sweep_fits(h) && h->launch.kernel != pplbm::kKernelTwoPass) {
        h->launch.kernel = pplbm::kKernelTwoPass;  // planes beyond 4 GiB: 64-bit plane offsets
        h->launch.tx = 256;
        h->launch.ty = 4;
    }
    return LBM_OK;
}

int lbm_strides(const lbm_t *h, size_t *row_stride, size_t *velocity_stride) {
    if (!h) return LBM_EINVAL;
    if (row_stride) *row_stride = h->p.frow;
    if (velocity_stride) *velocity_stride = h->p.fq;
    return LBM_OK;
}

int lbm_set_tile(lbm_t *h, int tx, int ty) {
    if (!h) return LBM_EINVAL;
    return lbm_set_launch(h, LBM_KERNEL_TWO_PASS, tx, ty, h->launch.flags);
}

int lbm_set_launch(lbm_t *h, int kernel, int tx, int ty, int flags) {
    if (!h) return LBM_EINVAL;
    if (flags & ~(LBM_LAUNCH_NONTEMPORAL | LBM_LAUNCH_XCD_ORDER | LBM_LAUNCH_SHALLOW))
        return fail(h, LBM_EINVAL, "unknown launch flags");
    if (kernel == LBM_KERNEL_TWO_PASS) {
        if (tx < 64 || tx % 64 || ty < 1 || tx * ty > 1024)
            return fail(h, LBM_EINVAL, "two-pass tile: tx a multiple of 64, ty >= 1, tx * ty <= 1024");
    } else if (kernel == LBM_KERNEL_SWEEP2) {
        if (tx < 64 || tx % 64 || tx > 256 || ty < 1)
            return fail(h, LBM_EINVAL, "two-step sweep: tx a multiple of 64 up to 256, ty >= 1 rows");
        if (!sweep_fits(h))
            return fail(h, LBM_EINVAL,
                        "two-step sweep: planes layout beyond 4 GiB (use the rows layout or the two-pass step)");
    } else if (kernel == LBM_KERNEL_SWEEP) {
        if (tx < 64 || tx % 64 || tx > 512 || ty < 1)
            return fail(h, LBM_EINVAL, "sweep: tx a multiple of 64 up to 512, ty >= 1 rows");
        if (!sweep_fits(h))
            return fail(h, LBM_EINVAL,
                        "sweep: planes layout beyond 4 GiB (use the rows layout or the two-pass step)");
    } else {
        return fail(h, LBM_EINVAL, "unknown kernel");
    }
    h->launch.kernel = kernel;
    h->launch.tx = tx;
    h->launch.ty = ty;
    h->launch.flags = flags;
    return LBM_OK;
}

int lbm_get_launch(const lbm_t *h, int *kernel, int *tx, int *ty, int *flags) {
    if (!h) return LBM_EINVAL;
    if (kernel) *kernel = h->launch.kernel;
    if (tx) *tx = h->launch.tx;
    if (ty) *ty = h->launch.ty;
    if (flags) *flags = h->launch.flags;
    return LBM_OK;
}

int lbm_set_probes(lbm_t *h, int xa, int ya, int xb, int yb) {
    if (!h) return LBM_EINVAL;
    if (xa < 0 || xa >= h->p.nx || xb < 0 || xb >= h->p.nx || ya < 0 || ya >= h->p.ny || yb < 0 ||
        yb >= h->p.ny)
        return fail(h, LBM_EINVAL, "probe outside the lattice");
    h->xa = xa;
    h->ya = ya;
    h->xb = xb;
    h->yb = yb;
    return LBM_OK;
}

int lbm_init(lbm_t *h, const double *rho0, const double *u0) {
    if (!h || !rho0) return LBM_EINVAL;
    const size_t N = (size_t)h->p.nx * h->p.ny;
    for (size_t k = 0; k < N; ++k) {
        const double eta = h->p.psi_kind == 0 ? h->eos.b * rho0[k] / 4.0 : 0.0;  // C-S packing limit
        if (!(rho0[k] > 0) || !(eta < 1)) return fail(h, LBM_EUNSTABLE, "initial density outside (0, 4/b)");
        if (u0 && (!std::isfinite(u0[2 * k]) || !std::isfinite(u0[2 * k + 1])))
            return fail(h, LBM_EINVAL, "non-finite initial velocity");
    }
    int rc = ensure_buffers(h);
    if (rc) return rc;
    double *d = nullptr;
    const size_t bytes = N * sizeof(double) * (u0 ? 3 : 1);
    if (hipMalloc(&d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, LBM_ENOMEM, "staging allocation failed");
    }
    hipError_t e = hipMemcpyAsync(d, rho0, N * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && u0)
        e = hipMemcpyAsync(d + N, u0, 2 * N * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = pplbm::launch_init(h->p, d, u0 ? d + N : nullptr, h->f[0], h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(h, e, "lbm_init");
    h->cur = 0;
    h->step = 0;
    h->initialised = true;
    h->vprev_valid = false;
    return LBM_OK;
}

// Three fresh timing events (folding the pending ones into the sums first if too many).
static int next_events(lbm *h, hipEvent_t **ev) {
    if (h->events_used >= 3 * kTimingFoldSteps) {
        int rc = fold_timing(h);
        if (rc) return rc;
    }
    if (h->events_used + 3 > h->events.size()) {
        for (int k = 0; k < 3 * 64; ++k) {
            hipEvent_t e;
            HIP_TRY(h, hipEventCreate(&e));
            h->events.push_back(e);
        }
    }
    *ev = &h->events[h->events_used];
    h->events_used += 3;
    return LBM_OK;
}

namespace {

// The launches of lbm_step.  *open is set while a timing triple is taken but its last event is
// not recorded yet.
static int step_launches(lbm *h, int n, bool *open) {
    const bool sweep2 = h->launch.kernel == pplbm::kKernelSweep2;
    const bool sweep = h->launch.kernel == pplbm::kKernelSweep || sweep2;
    // The sweep is timed per call, one pair of events around its n back-to-back launches: an
    // event between every two launches costs about 5 % of the step.  The two-pass step is
    // timed per step, to split the density/psi pass from the fused pass.
    hipEvent_t *call_ev = nullptr;
    if (h->timing && sweep && n > 0) {
        int rc = next_events(h, &call_ev);
        if (rc) return rc;
        *open = true;
        HIP_TRY(h, hipEventRecord(call_ev[0], h->stream));
        HIP_TRY(h, hipEventRecord(call_ev[1], h->stream));
    }
    int it = 0;
    if (sweep2) {  // pairs of steps in one launch each; an odd last step by the one-step sweep
        for (; it + 2 <= n; it += 2) {
            HIP_TRY(h, pplbm::launch_sweep2(h->p, h->prec, h->launch, h->f[h->cur],
                                            h->f[1 - h->cur], h->stream));
            h->cur = 1 - h->cur;
            h->step += 2;
        }
    }
    for (; it < n; ++it) {
        float *fc = h->f[h->cur], *fn = h->f[1 - h->cur];
        if (sweep2) {
            pplbm::Launch one = default_launch(h->p.nx, h->p.ny);
            HIP_TRY(h, pplbm::launch_sweep(h->p, h->prec, one, fc, fn, h->stream));
        } else if (sweep) {
            HIP_TRY(h, pplbm::launch_sweep(h->p, h->prec, h->launch, fc, fn, h->stream));
        } else {
            hipEvent_t *ev = nullptr;
            if (h->timing) {
                int rc = next_events(h, &ev);
                if (rc) return rc;
                *open = true;
                HIP_TRY(h, hipEventRecord(ev[0], h->stream));
            }
            HIP_TRY(h, pplbm::launch_psi(h->p, h->prec, h->launch.flags, fc, h->psi, h->stream));
            if (ev) HIP_TRY(h, hipEventRecord(ev[1], h->stream));
            HIP_TRY(h, pplbm::launch_fused(h->p, h->prec, h->launch, fc, h->psi, fn, h->stream));
            if (ev) {
                HIP_TRY(h, hipEventRecord(ev[2], h->stream));
                *open = false;
                ++h->timed_steps;
            }
        }
        h->cur = 1 - h->cur;
        ++h->step;
    }
    if (call_ev) {
        HIP_TRY(h, hipEventRecord(call_ev[2], h->stream));
        *open = false;
        h->timed_steps += n;
    }
    return LBM_OK;
}

}  // namespace

int lbm_step(lbm_t *h, int n) {
    if (!h || n < 0) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_step before lbm_init");
    bool open = false;
    const int rc = step_launches(h, n, &open);
    // a triple whose last event was never recorded is given back (it is always the last one
    // taken), so that folding the timings later does not wait on or read an unrecorded event
    if (open) h->events_used -= 3;
    return rc;
}

int lbm_autotune(lbm_t *h, const char *cache_path, int trial_steps, double *ms_out) {
    if (!h || trial_steps < 1) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_autotune before lbm_init");
    std::ostringstream key;
    key << pplbm::device_tag() << "|single|" << h->p.nx << "x" << h->p.ny << "|scheme" << h->p.scheme
        << "|coll" << h->p.coll << "|prec" << h->prec << "|layout" << h->layout;
    std::string hit;
    if (pplbm::tune_cache_lookup(cache_path, key.str(), &hit)) {
        int k = 0, tx = 0, ty = 0, fl = 0;
        if (std::sscanf(hit.c_str(), "%d %d %d %d", &k, &tx, &ty, &fl) == 4 &&
            lbm_set_launch(h, k, tx, ty, fl) == LBM_OK) {
            if (ms_out) *ms_out = -1.0;  // from the cache, not timed now
            return LBM_OK;
        }
    }
    // Trials run on the current state; it is saved first and restored afterwards.
    const size_t fbytes = 9 * h->p.plane * sizeof(float);
    float *saved = nullptr;
    if (hipMalloc(&saved, fbytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, LBM_ENOMEM, "autotune: state copy allocation failed");
    }
    const int cur0 = h->cur;
    const long long step0 = h->step;
    const bool timing0 = h->timing;  // steps leave vprev alone, so its snapshot stays valid
    const pplbm::Launch before = h->launch;
    h->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LBM_OK;
    hipError_t he = hipMemcpyAsync(saved, h->f[cur0], fbytes, hipMemcpyDeviceToDevice, h->stream);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    pplbm::Launch best = before;
    double best_ms = 1e300;
    // one timed trial of a shape (an even number of steps, so both kernels compare per step)
    const int nsteps = trial_steps + (trial_steps & 1);
    auto trial = [&](int kernel, int tx, int ty, int fl) {
        rc = lbm_set_launch(h, kernel, tx, ty, fl);
        if (!rc) rc = lbm_step(h, 2);  // warm-up (first-launch costs)
        if (rc) return;
        he = hipEventRecord(e0, h->stream);
        if (he == hipSuccess) rc = lbm_step(h, nsteps);
        if (he == hipSuccess && !rc) he = hipEventRecord(e1, h->stream);
        if (he == hipSuccess && !rc) he = hipEventSynchronize(e1);
        float ms = 0;
        if (he == hipSuccess && !rc) he = hipEventElapsedTime(&ms, e0, e1);
        if (he == hipSuccess && !rc && ms / nsteps < best_ms) {
            best_ms = ms / nsteps;
            best = h->launch;
        }
    };
    const int txs[] = {64, 128, 256, 512};
    const int tys[] = {4, 8, 16, 32, 64};
    const int fls[] = {pplbm::kFlagXCD | pplbm::kFlagShallow, pplbm::kFlagShallow,
                       pplbm::kFlagXCD, pplbm::kFlagXCD | pplbm::kFlagShallow | pplbm::kFlagNT};
    const int width = (int)std::min<size_t>(h->p.pitch, 512);
    if (sweep_fits(h)) {
        for (int tx : txs) {
            if (tx > 64 && tx > width) continue;  // strips wider than the lattice only idle
            for (int ty : tys) {
                if (ty > 8 && ty / 2 >= h->p.ny) continue;
                for (int fl : fls) {
                    if (he != hipSuccess || rc) break;
                    trial(LBM_KERNEL_SWEEP, tx, ty, fl);
                }
            }
        }
        for (int tx : {64, 128, 256})  // two steps per launch
            for (int ty : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32})
                for (int fl : {pplbm::kFlagXCD, 0}) {
                    if (he != hipSuccess || rc) break;
                    if (ty > 6 && ty / 2 >= h->p.ny) continue;
                    trial(LBM_KERNEL_SWEEP2, tx, ty, fl);
                }
    } else {  // planes layout beyond 4 GiB: only the two-pass step can run
        for (int tx : {64, 128, 256})
            for (int ty : {2, 4, 8}) {
                if (he != hipSuccess || rc) break;
                if (tx * ty > 1024) continue;  // threads per workgroup of the fused pass
                trial(LBM_KERNEL_TWO_PASS, tx, ty, pplbm::kFlagXCD);
            }
    }
    // restore the state whatever happened
    hipError_t he2 = hipMemcpyAsync(h->f[cur0], saved, fbytes, hipMemcpyDeviceToDevice, h->stream);
    if (he2 == hipSuccess) he2 = hipStreamSynchronize(h->stream);
    (void)hipFree(saved);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    h->cur = cur0;
    h->step = step0;
    h->timing = timing0;
    if (he != hipSuccess) {
        h->launch = before;
        return hip_fail(h, he, "autotune trial");
    }
    if (he2 != hipSuccess) return hip_fail(h, he2, "autotune restore");
    if (rc) {
        h->launch = before;
        return rc;
    }
    h->launch = best;
    std::ostringstream val;
    val << best.kernel << " " << best.tx << " " << best.ty << " " << best.flags;
    pplbm::tune_cache_store(cache_path, key.str(), val.str(), best_ms);
    if (ms_out) *ms_out = best_ms;
    return LBM_OK;
}

int lbm_read(lbm_t *h, double *rho, double *u) {
    if (!h) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_read before lbm_init");
    const size_t N = (size_t)h->p.nx * h->p.ny;
    double *d = nullptr;
    if (hipMalloc(&d, 3 * N * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, LBM_ENOMEM, "staging allocation failed");
    }
    float *fc = h->f[h->cur];
    hipError_t e = pplbm::launch_psi(h->p, pplbm::kPrecF64, 0, fc, h->psi, h->stream);
    if (e == hipSuccess) e = pplbm::launch_macro(h->p, fc, h->psi, d, d + N, h->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, d + N, 2 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(h, e, "lbm_read");
    return LBM_OK;
}

// Checkpoint file: "PPLBMCK1", int32 nx, ny, int64 step, the parameter structs as written by
// this library (eos, force, collision, tau), then FP32 populations [9][ny][nx].
namespace {
constexpr char kCkptMagic[8] = {'P', 'P', 'L', 'B', 'M', 'C', 'K', '1'};

// Field by field (the structs have padding).
static bool same_params(const lbm_eos &a, const lbm_eos &b, const lbm_force &fa, const lbm_force &fb,
                        const lbm_collision &ca, const lbm_collision &cb) {
    return a.kind == b.kind && a.a == b.a && a.b == b.b && a.R == b.R && a.T_over_Tc == b.T_over_Tc &&
           a.K == b.K && a.eps == b.eps && fa.scheme == fb.scheme && fa.A == fb.A &&
           fa.sigma == fb.sigma && fa.G == fb.G && ca.kind == cb.kind && ca.s_rho == cb.s_rho &&
           ca.s_e == cb.s_e && ca.s_eps == cb.s_eps && ca.s_j == cb.s_j && ca.s_q == cb.s_q;
}
}  // namespace

int lbm_save(lbm_t *h, const char *path) {
    if (!h || !path) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_save before lbm_init");
    const size_t n = 9 * (size_t)h->p.nx * h->p.ny;
    std::vector<float> f;
    try {
        f.resize(n);
    } catch (...) {
        return fail(h, LBM_ENOMEM, "checkpoint staging buffer");
    }
    int rc = lbm_populations(h, f.data());
    if (rc) return rc;
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return fail(h, LBM_EINVAL, std::string("cannot open ") + path);
    const int32_t dims[2] = {h->p.nx, h->p.ny};
    const int64_t step = h->step;
    bool ok = std::fwrite(kCkptMagic, 1, 8, fp) == 8 && std::fwrite(dims, sizeof dims, 1, fp) == 1 &&
              std::fwrite(&step, sizeof step, 1, fp) == 1 &&
              std::fwrite(&h->eos, sizeof h->eos, 1, fp) == 1 &&
              std::fwrite(&h->force, sizeof h->force, 1, fp) == 1 &&
              std::fwrite(&h->coll, sizeof h->coll, 1, fp) == 1 &&
              std::fwrite(&h->tau, sizeof h->tau, 1, fp) == 1 &&
              std::fwrite(f.data(), sizeof(float), n, fp) == n;
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? LBM_OK : fail(h, LBM_EINVAL, std::string("write failed: ") + path);
}

int lbm_load(lbm_t *h, const char *path) {
    if (!h || !path) return LBM_EINVAL;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return fail(h, LBM_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    int32_t dims[2];
    int64_t step = 0;
    lbm_eos eos;
    lbm_force force;
    lbm_collision coll;
    double tau = 0;
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, kCkptMagic, 8) == 0 &&
              std::fread(dims, sizeof dims, 1, fp) == 1 && std::fread(&step, sizeof step, 1, fp) == 1 &&
              std::fread(&eos, sizeof eos, 1, fp) == 1 && std::fread(&force, sizeof force, 1, fp) == 1 &&
              std::fread(&coll, sizeof coll, 1, fp) == 1 && std::fread(&tau, sizeof tau, 1, fp) == 1;
    if (!ok) {
        std::fclose(fp);
        return fail(h, LBM_EINVAL, "not a checkpoint of this library");
    }
    if (dims[0] != h->p.nx || dims[1] != h->p.ny ||
        !same_params(eos, h->eos, force, h->force, coll, h->coll) || tau != h->tau) {
        std::fclose(fp);
        return fail(h, LBM_EINVAL, "checkpoint of another lattice (size or parameters differ)");
    }
    const size_t n = 9 * (size_t)h->p.nx * h->p.ny;
    std::vector<float> f;
    try {
        f.resize(n);
    } catch (...) {
        std::fclose(fp);
        return fail(h, LBM_ENOMEM, "checkpoint staging buffer");
    }
    ok = std::fread(f.data(), sizeof(float), n, fp) == n;
    std::fclose(fp);
    if (!ok) return fail(h, LBM_EINVAL, "truncated checkpoint");
    int rc = lbm_set_populations(h, f.data());
    if (rc) return rc;
    h->step = step;
    return LBM_OK;
}

int lbm_populations(lbm_t *h, float *f) {
    if (!h || !f) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_populations before lbm_init");
    const Physics &p = h->p;
    const float *src = h->f[h->cur];
    for (int q = 0; q < 9; ++q)
        HIP_TRY(h, hipMemcpy2DAsync(f + (size_t)q * p.nx * p.ny, p.nx * sizeof(float),
                                    src + q * p.fq, p.frow * sizeof(float), p.nx * sizeof(float),
                                    p.ny, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_set_populations(lbm_t *h, const float *f) {
    if (!h || !f) return LBM_EINVAL;
    int rc = ensure_buffers(h);
    if (rc) return rc;
    const Physics &p = h->p;
    float *dst = h->f[h->cur];
    for (int q = 0; q < 9; ++q)
        HIP_TRY(h, hipMemcpy2DAsync(dst + q * p.fq, p.frow * sizeof(float),
                                    f + (size_t)q * p.nx * p.ny, p.nx * sizeof(float),
                                    p.nx * sizeof(float), p.ny, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->initialised = true;
    h->vprev_valid = false;
    return LBM_OK;
}

// lbm_stats_t from the reduction's result vector (sum, min, max, max |v|, max |dv|,
// non-finite count, probe a, probe b); dv_max only when a previous velocity was kept.
static int fill_stats(lbm *h, const double r[pplbm::kStatsOut], bool dv, lbm_stats_t *out) {
    out->mass = r[0];
    out->rho_min = r[1];
    out->rho_max = r[2];
    out->us_max = r[3];
    out->dv_max = dv ? r[4] : 0.0;
    out->nonfinite = (int)r[5];
    out->rho_probe_a = r[6];
    out->rho_probe_b = r[7];
    const double hi = std::fmax(r[6], r[7]), lo = std::fmin(r[6], r[7]);
    out->ratio = hi / lo;
    out->step = h->step;
    if (out->nonfinite) return fail(h, LBM_EUNSTABLE, "non-finite or undefined state at some node");
    return LBM_OK;
}

int lbm_stats(lbm_t *h, int track_dv, lbm_stats_t *out) {
    if (!h || !out) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_stats before lbm_init");
    int rc = ensure_stats(h);
    if (rc) return rc;
    const size_t N = (size_t)h->p.nx * h->p.ny;
    if (track_dv && !h->vprev) {
        if (hipMalloc(&h->vprev, 2 * N * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, LBM_ENOMEM, "allocation of the velocity history failed");
        }
        h->vprev_valid = false;
    }
    float *fc = h->f[h->cur];
    HIP_TRY(h, pplbm::launch_psi(h->p, pplbm::kPrecF64, 0, fc, h->psi, h->stream));
    HIP_TRY(h, pplbm::launch_stats(h->p, fc, h->psi, track_dv ? h->vprev : nullptr, h->stats_partial,
                                   h->stats_out, h->xa, h->ya, h->xb, h->yb, h->stream));
    double r[pplbm::kStatsOut];
    HIP_TRY(h, hipMemcpyAsync(r, h->stats_out, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const bool dv = track_dv && h->vprev_valid;
    if (track_dv) h->vprev_valid = true;
    return fill_stats(h, r, dv, out);
}

int lbm_stats_noalloc(lbm_t *h, lbm_stats_t *out) {
    if (!h || !out) return LBM_EINVAL;
    if (!h->initialised) return fail(h, LBM_ESTATE, "lbm_stats_noalloc before lbm_init");
    double *scr = nullptr;
    size_t cap = 0;
    HIP_TRY(h, pplbm::stats_scratch(&scr, &cap));
    const size_t parts = pplbm::stats_partial_count(h->p) * pplbm::kStatsFields;
    if (parts + pplbm::kStatsOut > cap)
        return fail(h, LBM_EINVAL, "lbm_stats_noalloc: the reduction needs more partials than "
                                   "the library's fixed device array holds");
    float *fc = h->f[h->cur];
    HIP_TRY(h, pplbm::launch_psi(h->p, pplbm::kPrecF64, 0, fc, h->psi, h->stream));
    HIP_TRY(h, pplbm::launch_stats(h->p, fc, h->psi, nullptr, scr, scr + parts, h->xa, h->ya,
                                   h->xb, h->yb, h->stream));
    double r[pplbm::kStatsOut];
    HIP_TRY(h, hipMemcpyAsync(r, scr + parts, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return fill_stats(h, r, false, out);
}

int lbm_timing_enable(lbm_t *h, int enable) {
    if (!h) return LBM_EINVAL;
    h->timing = enable != 0;
    return LBM_OK;
}

int lbm_timing(lbm_t *h, double *psi_ms, double *fused_ms, long long *steps) {
    if (!h) return LBM_EINVAL;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    int rc = fold_timing(h);
    if (rc) return rc;
    if (psi_ms) *psi_ms = h->timed_a;
    if (fused_ms) *fused_ms = h->timed_b;
    if (steps) *steps = h->timed_steps;
    h->timed_a = h->timed_b = 0.0;
    h->timed_steps = 0;
    return LBM_OK;
}

int lbm_eos_critical(const lbm_eos *eos, double *rho_c, double *T_c, double *p_c) {
    if (!eos || eos->kind != LBM_EOS_CARNAHAN_STARLING) return LBM_EINVAL;
    if (!(eos->a > 0) || !(eos->b > 0) || !(eos->R > 0)) return LBM_EINVAL;
    critical(eos->a, eos->b, eos->R, rho_c, T_c, p_c);
    return LBM_OK;
}

int lbm_eos_maxwell(const lbm_eos *eos, double *rho_g, double *rho_l) {
    if (!eos || eos->kind != LBM_EOS_CARNAHAN_STARLING) return LBM_EINVAL;
    if (!rho_g || !rho_l || !(eos->a > 0) || !(eos->b > 0) || !(eos->R > 0)) return LBM_EINVAL;
    if (!(eos->T_over_Tc > 0 && eos->T_over_Tc < 1)) return LBM_EINVAL;
    return maxwell(*eos, rho_g, rho_l);
}

const char *lbm_strerror(int code) {
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EUNSTABLE: return "unstable state";
    case LBM_ENOTCONVERGED: return "not converged";
    case LBM_ESTATE: return "call out of order";
    default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_t *h) { return h ? h->err.c_str() : ""; }

int lbm_copy_f32(float *dst, const float *src, size_t n, void *stream) {
    if (!dst || !src) return LBM_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) & 15) return LBM_EINVAL;
    return pplbm::launch_copy(dst, src, n, (hipStream_t)stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

}  // extern "C"
