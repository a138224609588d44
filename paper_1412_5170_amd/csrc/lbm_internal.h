// Internal interface between the C ABI runtime (lbm_api.cpp) and the gfx950 kernels
// (lbm_kernels.hip).  Not installed; the public interface is include/pplbm.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "../../include/pplbm.h"

namespace pplbm {

enum Scheme { EDM = 0, GUO = 1, GUO_LI = 2, SC = 3 };
enum Coll { BGK = 0, MRT = 1 };

// Everything a step needs, in FP64; the launchers convert to the kernels' arithmetic type.
struct Physics {
    int nx, ny;
    size_t pitch;   // floats per row of the psi plane (multiple of 64, >= nx)
    size_t plane;   // floats per population plane (pitch * ny)
    size_t frow;    // population row stride: pitch (planes layout) or 9 * pitch (rows layout)
    size_t fq;      // population velocity stride: plane (planes layout) or pitch (rows layout)
    double b_quarter;   // b / 4                     (Eq. 29)
    double RT;          // R * T                     (Eq. 29)
    double a;           // attraction constant       (Eq. 29)
    double K;           // EOS rescale               (Eq. 30)
    double G;           // interaction strength      (Eq. 4-7), < 0
    double A;           // hybrid weight             (Eq. 6)
    double sigma;       // Li's constant             (Eq. 31)
    double tau;         // relaxation time           (Eq. 1)
    int psi_kind;       // 0: psi from the EOS (Eq. 7); 1: psi of Eq. 33
    double inv_eps;     // Eq. 33: 1/eps, 0 for the exp(-1/rho) form
    double s[9];        // MRT rates, moment order (rho, e, eps, jx, qx, jy, qy, pxx, pxy)
    int scheme, coll;
};

enum { kPrecF64 = 1, kPrecMixed = 2 };  // the values of LBM_PREC_*

// The kernel a lattice runs, as scheme * 2 + collision: the exact-difference and Shan-Chen
// schemes with BGK, Guo's schemes (with or without Li's term) with the moment-space collision
// that serves BGK (every rate 1/tau) and MRT alike, so both collisions share one kernel.
inline int kernel_kind(int scheme) {
    return scheme == GUO || scheme == GUO_LI ? scheme * 2 + MRT : scheme * 2 + BGK;
}
constexpr int kFlagNT = 1;   // non-temporal stores of the new populations
constexpr int kFlagXCD = 2;  // XCD-aware order of the tiles
constexpr int kFlagShallow = 4;  // sweep: prefetch one row ahead instead of two
enum { kKernelTwoPass = 0, kKernelSweep = 1, kKernelSweep2 = 2 };

// Segment height of a two-step sweep launch from its wave count W(H) (strips of 58 output
// columns x segments of H rows, summed over the lattices the launch covers).  Many waves: 16
// rows where W(16) >= 8192, else 24 where W(24) >= 3072, else the lowest height from 6 rows up
// with W <= 3200 (one resident round: 4096 wave slots).  Where that is 6 rows the launch cannot
// fill the GPU and takes as long as its busiest SIMD: about (H + 4) rows of iterations times
// max(1.5, ceil(W(H) / 1024)) (waves per SIMD; a lone wave issues at about two thirds of the
// rate of two or more), minimised over H in 1..12 (the larger H on a tie).  Sets *small when
// the latter rule decided.
template <typename F>
int two_step_height(F waves, bool *small = nullptr) {
    if (small) *small = false;
    if (waves(16) >= 8192) return 16;
    if (waves(24) >= 3072) return 24;
    int h = 24;
    for (int rows = 6; rows < 24; ++rows)
        if (waves(rows) <= 3200) {
            h = rows;
            break;
        }
    if (h > 6) return h;
    long long best = -1;
    for (int rows = 1; rows <= 12; ++rows) {
        const long long k = ((long long)waves(rows) + 1023) / 1024;
        const long long cost = (rows + 4) * (k < 2 ? 3 : 2 * k);  // 2 (H + 4) max(1.5, k)
        if (best < 0 || cost <= best) {
            best = cost;
            h = rows;
        }
    }
    if (small) *small = true;
    return h;
}

// Shape of the step launch.  Two-pass: (tx, ty) is the fused pass's tile.  Sweep: tx columns
// per workgroup, ty rows per segment.
struct Launch {
    int kernel = kKernelTwoPass;
    int tx = 64, ty = 4;
    int flags = 0;
};

// Validated physics of one lattice (rows layout); T_out receives the absolute temperature.
int make_physics(int nx, int ny, const lbm_eos *eos, const lbm_force *force,
                 const lbm_collision *collision, double tau, Physics *out, double *T_out,
                 std::string *why);

// Density / psi pass (Eq. 3, Eq. 29-30, Eq. 7): psi[y * pitch + x] from f.
hipError_t launch_psi(const Physics &p, int prec, int flags, const float *f, float *psi,
                      hipStream_t stream);

// Fused pass: force (Eq. 6) + forcing scheme + BGK/MRT collision + push streaming (Eq. 36).
hipError_t launch_fused(const Physics &p, int prec, const Launch &L, const float *fin,
                        const float *psi, float *fout, hipStream_t stream);

// Whole step in one pass (psi recomputed from f along a sweep): fin -> fout.
hipError_t launch_sweep(const Physics &p, int prec, const Launch &L, const float *fin,
                        float *fout, hipStream_t stream);
// Two time steps per launch (temporal blocking); L.tx threads per workgroup (64-lane
// independent strips), L.ty rows per segment.  Populations below 4 GiB.
hipError_t launch_sweep2(const Physics &p, int prec, const Launch &L, const float *fin,
                         float *fout, hipStream_t s);

// f = f^eq(rho0, u0) (Eq. 2); rho0 [ny*nx], u0 [ny*nx*2] or null, device FP64.
// Radial-profile initial state: log_rho holds 64 values (host memory, passed by value).
int profile_mass_blocks(const Physics &p);
hipError_t launch_profile_mass(const Physics &p, const double *log_rho, double r0, double dr,
                               double shift, double *partial, hipStream_t s);
hipError_t launch_profile_init(const Physics &p, const double *log_rho, double r0, double dr,
                               double shift, float *f, hipStream_t s);
// f (holding f^eq(rho, 0)) -> f^eq(rho, -F / (2 rho)) in place; psi: a scratch psi plane.
hipError_t launch_rest(const Physics &p, float *f, float *psi, hipStream_t s);
hipError_t launch_init(const Physics &p, const double *rho0, const double *u0, float *f,
                       hipStream_t stream);

// rho and v = u + F/(2 rho) into device FP64 arrays (compact, x fastest); needs a psi pass
// on the same f first.
hipError_t launch_macro(const Physics &p, const float *f, const float *psi, double *rho,
                        double *u, hipStream_t stream);

// Deterministic FP64 reduction of the observables.  partial must hold
// stats_partial_count(p) * kStatsFields doubles, out kStatsOut doubles.  vprev (2 floats per
// node, pitch layout) may be null; when given, dv is measured against it and it is updated.
constexpr int kStatsFields = 6;  // sum rho, min rho, max rho, max |v|, max |dv|, nonfinite
constexpr int kStatsOut = 8;     // the six above + rho at probe a, rho at probe b
size_t stats_partial_count(const Physics &p);
hipError_t launch_stats(const Physics &p, const float *f, const float *psi, float *vprev,
                        double *partial, double *out, int xa, int ya, int xb, int yb,
                        hipStream_t stream);

// The library's fixed device array for the allocation-free observables on the current device:
// *ptr receives its device address (looked up once per device), *doubles its length.
hipError_t stats_scratch(double **ptr, size_t *doubles);

hipError_t launch_copy(float *dst, const float *src, size_t n, hipStream_t stream);

// ---- batched sweep ----------------------------------------------------------------------
// Device descriptor of one batch lattice (opaque to the runtime; filled on the host).
size_t batch_lattice_bytes();
void batch_lattice_fill(const Physics &p, float *f0, float *f1, float *vprev, int xa, int ya,
                        int xb, int yb, int flags, void *out);
// One step of the batch lattices of one kind (`scheme`, `coll`; `kind` indexes meta): the tiles
// tiles[meta[kind].x + t] = (lattice, x0, y0, rows), t < meta[kind].y, read from f[parity] and
// written to f[parity ^ 1]; tx threads per workgroup, `groups` persistent workgroups.
hipError_t launch_batch_kind(const void *lats, const int4 *tiles, const int2 *meta, int kind,
                             int scheme, int coll, int parity, int tx, int groups, bool shallow,
                             hipStream_t s);

// Two steps of one kind of the batch (f[parity] -> f[parity ^ 1]): groups workgroups of four
// independent waves walk the kind's slice of the two-step tile list (lattice, first output
// column, first row, rows), each tile a strip of sweep2_out_columns() output columns.
hipError_t launch_batch2_kind(const void *lats, const int4 *tiles, const int2 *meta, int kind,
                              int scheme, int coll, int parity, int groups, hipStream_t s);
int sweep2_out_columns();

// Observables of the lattices listed in ids (nlat of them) from f[parity]: sblocks[b] =
// (lattice, chunk, chunks, partial slot); ranges[i] = (first partial, count) of ids[i]; out
// receives kStatsOut doubles per lattice id.
hipError_t launch_batch_stats(const void *lats, const int4 *sblocks, int nsblocks,
                              const int2 *ranges, const int *ids, int nlat, int parity, int track,
                              double *partial, double *out, hipStream_t stream);

// Bytes of one population buffer (9 velocity planes).  Up to kSweepMaxBytes the one-pass
// sweep addresses it through one buffer resource with 32-bit offsets; beyond, through one
// resource per row (rows layout only).  The batch's lattices stay below it.
inline size_t pop_bytes(const Physics &p) { return 9 * p.plane * sizeof(float); }
constexpr size_t kSweepMaxBytes = 0xFFFFFFFFull;

// Exact critical point of Eq. 29 (dp/drho = d2p/drho2 = 0), host.
void critical_point(double a, double b, double R, double *rho_c, double *T_c, double *p_c);

// Autotuner cache (JSON lines; see lbm_tune.cpp).
std::string device_tag();
bool tune_cache_lookup(const char *path, const std::string &key, std::string *value);
bool tune_cache_store(const char *path, const std::string &key, const std::string &value, double ms);

}  // namespace pplbm
