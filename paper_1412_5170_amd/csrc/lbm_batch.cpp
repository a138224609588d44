// Batched sweep runtime (include/pplbm.h, lbm_batch_*): many independent periodic lattices --
// each with its own size, EOS temperature and rescale, forcing, collision and relaxation time --
// advanced together, one launch per time step over a shared device tile list; blocks of steps
// are captured once in a hipGraph and replayed; FP64 observables per lattice at every check;
// converged or unstable lattices are dropped from the tile list in device memory between
// replays, so the captured graph stays valid.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pplbm.h"
#include "lbm_internal.h"

using pplbm::Physics;

struct lbm_batch {
    int count = 0;
    std::vector<Physics> phys;
    std::vector<lbm_eos> eos;        // as given (Maxwell densities of the plain start)
    std::vector<lbm_force> force;
    std::vector<float *> f0, f1, vprev;
    std::vector<int> seg_rows;       // segment height of each lattice's tiles (0: automatic)
    int auto_rows = 32;              // segment height of the automatic lattices, per upload
    std::vector<char> active;
    std::vector<char> initialised;
    std::vector<long long> steps;
    std::vector<char> vprev_valid;
    std::vector<int> xa, ya, xb, yb;
    void *desc = nullptr;            // device BatchLattice[count]
    int4 *tiles = nullptr;           // device tile list (capacity max_tiles)
    int2 *meta = nullptr;            // device (offset, count) of each kind's tiles
    int4 *tiles2 = nullptr;          // two-step tile list: (lattice, first output column,
    int2 *meta2 = nullptr;           //   first row, rows), and each kind's slice of it
    size_t max_tiles2 = 0;
    int rows2 = 24;                  // segment height of the two-step tiles, per upload
    std::vector<int> kind_tiles2;    // two-step tiles of each kind, per upload
    std::vector<int> graph_tiles2;   // the same when the graph was captured (its grid sizes)
    std::vector<int> kinds;          // kernel kinds present (pplbm::kernel_kind), ascending
    size_t max_tiles = 0;
    // observables
    int4 *sblocks = nullptr;
    int2 *ranges = nullptr;
    int *ids = nullptr;
    double *partial = nullptr, *out = nullptr;
    size_t max_sblocks = 0;
    // launch
    // two steps per launch; one-step launches (the rest of a 2 mod 4 step count) with
    // 256-column strips and two rows of loads in flight
    int tx = 256, groups = 0, flags = LBM_LAUNCH_TWO_STEP;
    hipStream_t stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_steps = 0;
    bool tiles_dirty = true;
    std::string err;
};

namespace {

int bfail(lbm_batch *b, int code, const std::string &m) {
    if (b) b->err = m;
    return code;
}

#define BHIP(b, call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) return bfail(b, LBM_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// Destroys the captured graph once no launch of it can still be running (the autotuner
// alternates graphs of 2 and trial_steps steps back to back).
void drop_graph(lbm_batch *b) {
    if (!b->graph) return;
    (void)hipStreamSynchronize(b->stream);
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

constexpr int kAutoRowsMax = 32, kAutoRowsMin = 4;
constexpr size_t kAutoTiles = 4096;  // ~16 workgroups per compute unit

size_t tiles_at(const lbm_batch *b, int i, int rows) {
    const Physics &p = b->phys[i];
    return (size_t)((p.nx + b->tx - 1) / b->tx) * ((p.ny + rows - 1) / rows);
}

// Most tiles lattice i can ever have (capacity of the device tile list).
size_t tiles_max(const lbm_batch *b, int i) {
    return tiles_at(b, i, b->seg_rows[i] ? b->seg_rows[i] : kAutoRowsMin);
}


size_t tiles2_at(const lbm_batch *b, int i, int rows) {
    const Physics &p = b->phys[i];
    const int w = pplbm::sweep2_out_columns();
    return (size_t)((p.nx + w - 1) / w) * ((p.ny + rows - 1) / rows);
}

// Segment height of the two-step tiles of the active lattices: the single lattice's rule
// (two_step_height) on the total wave count, the kinds running one after another.  As converged
// lattices leave, the ones still running are cut into shorter segments, so the last few still
// spread over the GPU.
int two_step_rows(const lbm_batch *b) {
    return pplbm::two_step_height([&](int rows) {
        size_t n = 0;
        for (int i = 0; i < b->count; ++i)
            if (b->active[i]) n += tiles2_at(b, i, rows);
        return (long long)n;
    });
}

bool two_step(const lbm_batch *b) { return b->flags & LBM_LAUNCH_TWO_STEP; }

int upload_desc(lbm_batch *b) {
    const size_t sz = pplbm::batch_lattice_bytes();
    std::vector<char> host(sz * b->count);
    for (int i = 0; i < b->count; ++i)
        pplbm::batch_lattice_fill(b->phys[i], b->f0[i], b->f1[i], b->vprev[i], b->xa[i], b->ya[i],
                                  b->xb[i], b->yb[i], b->flags & pplbm::kFlagNT, host.data() + i * sz);
    BHIP(b, hipMemcpyAsync(b->desc, host.data(), host.size(), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

// Tile list of the active lattices (strips of tx columns x segments of rows).  Lattices with
// an automatic segment height share one, halved from 32 down to 4 rows until the active tiles
// number about 4096: as converged lattices leave, the ones still running are cut finer, so a
// lone large lattice still spreads over every compute unit.  (Tile shapes do not change the
// results, which are bitwise those of any other shape.)
int upload_tiles(lbm_batch *b) {
    size_t need = 0;
    for (int i = 0; i < b->count; ++i) need += tiles_max(b, i);
    if (need > b->max_tiles) {
        drop_graph(b);  // the captured graph holds the old tile list pointer; let it finish
        if (b->tiles) (void)hipFree(b->tiles);
        b->tiles = nullptr;
        b->max_tiles = 0;
        if (hipMalloc(&b->tiles, need * sizeof(int4)) != hipSuccess) {
            (void)hipGetLastError();
            return bfail(b, LBM_ENOMEM, "tile list allocation failed");
        }
        b->max_tiles = need;
    }
    b->auto_rows = kAutoRowsMax;
    for (;;) {
        size_t n = 0;
        for (int i = 0; i < b->count; ++i)
            if (b->active[i]) n += tiles_at(b, i, b->seg_rows[i] ? b->seg_rows[i] : b->auto_rows);
        if (n >= kAutoTiles || b->auto_rows <= kAutoRowsMin) break;
        b->auto_rows /= 2;
    }
    std::vector<int4> t;
    t.reserve(need);
    std::vector<int2> meta;
    for (int kind : b->kinds) {  // tiles grouped by kind, one slice per kind
        const int first = (int)t.size();
        for (int i = 0; i < b->count; ++i) {
            if (!b->active[i]) continue;
            const Physics &p = b->phys[i];
            if (pplbm::kernel_kind(p.scheme) != kind) continue;
            const int H = b->seg_rows[i] ? b->seg_rows[i] : b->auto_rows;
            for (int y0 = 0; y0 < p.ny; y0 += H)
                for (int x0 = 0; x0 < p.nx; x0 += b->tx) t.push_back(make_int4(i, x0, y0, H));
        }
        meta.push_back(make_int2(first, (int)t.size() - first));
    }
    if (!t.empty())
        BHIP(b, hipMemcpyAsync(b->tiles, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->meta, meta.data(), meta.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    // the two-step tiles of the active lattices, grouped by kind in the same order
    std::vector<int4> t2;
    std::vector<int2> meta2;
    if (two_step(b)) {
        b->rows2 = two_step_rows(b);
        size_t need2 = 0;
        for (int i = 0; i < b->count; ++i)
            if (b->active[i]) need2 += tiles2_at(b, i, b->rows2);
        if (need2 > b->max_tiles2) {
            drop_graph(b);
            if (b->tiles2) (void)hipFree(b->tiles2);
            b->tiles2 = nullptr;
            b->max_tiles2 = 0;
            if (hipMalloc(&b->tiles2, need2 * sizeof(int4)) != hipSuccess) {
                (void)hipGetLastError();
                return bfail(b, LBM_ENOMEM, "two-step tile list allocation failed");
            }
            b->max_tiles2 = need2;
        }
        const int w = pplbm::sweep2_out_columns();
        for (int kind : b->kinds) {
            const int first = (int)t2.size();
            for (int i = 0; i < b->count; ++i) {
                if (!b->active[i]) continue;
                const Physics &p = b->phys[i];
                if (pplbm::kernel_kind(p.scheme) != kind) continue;
                for (int y0 = 0; y0 < p.ny; y0 += b->rows2)
                    for (int x0 = 0; x0 < p.nx; x0 += w) t2.push_back(make_int4(i, x0, y0, b->rows2));
            }
            meta2.push_back(make_int2(first, (int)t2.size() - first));
        }
        b->kind_tiles2.clear();
        for (const int2 &m : meta2) b->kind_tiles2.push_back(m.y);
        if (!t2.empty())
            BHIP(b, hipMemcpyAsync(b->tiles2, t2.data(), t2.size() * sizeof(int4), hipMemcpyHostToDevice,
                                   b->stream));
        BHIP(b, hipMemcpyAsync(b->meta2, meta2.data(), meta2.size() * sizeof(int2), hipMemcpyHostToDevice,
                               b->stream));
    }
    BHIP(b, hipStreamSynchronize(b->stream));
    b->tiles_dirty = false;
    return LBM_OK;
}

int grid_groups(const lbm_batch *b) {
    if (b->groups > 0) return std::max(b->groups / 8 * 8, 8);
    size_t all = 0;
    for (int i = 0; i < b->count; ++i) all += tiles_max(b, i);
    size_t g = std::min<size_t>(all, 2048);  // ~8 workgroups per compute unit
    g = std::max<size_t>(g / 8 * 8, 8);      // a multiple of 8: each XCD walks its own eighth
    return (int)g;
}

// Workgroups (of four waves) of a two-step launch of kind j: one wave per tile of the current
// tile list, so the hardware hands tiles to free wave slots as they come.  The graph is
// captured again whenever these counts change.
int grid2_groups(const lbm_batch *b, size_t j) {
    const int n = j < b->kind_tiles2.size() ? b->kind_tiles2[j] : 0;
    return std::max(1, (n + 3) / 4);
}

// n (even) steps as launches: with two steps per launch, 2 (n / 4) two-step launches and the
// rest (0 or 2) one-step launches, an even number of buffer swaps in all, so every lattice's
// populations are back in f[0] after the n steps, as with n one-step launches.
void step_plan(const lbm_batch *b, int n, int *two, int *one) {
    *two = two_step(b) ? 2 * (n / 4) : 0;
    *one = n - 2 * *two;
}

hipError_t launch_kind(lbm_batch *b, size_t j, bool two, int parity, hipStream_t s) {
    if (two)
        return pplbm::launch_batch2_kind(b->desc, b->tiles2, b->meta2, (int)j, b->kinds[j] / 2,
                                         b->kinds[j] % 2, parity, grid2_groups(b, j), s);
    return pplbm::launch_batch_kind(b->desc, b->tiles, b->meta, (int)j, b->kinds[j] / 2,
                                    b->kinds[j] % 2, parity, b->tx, grid_groups(b),
                                    b->flags & pplbm::kFlagShallow, s);
}

int launch_steps(lbm_batch *b, int n) {
    int two, one;
    step_plan(b, n, &two, &one);
    int parity = 0;
    for (int k = 0; k < two + one; ++k, parity ^= 1)
        for (size_t j = 0; j < b->kinds.size(); ++j)
            BHIP(b, launch_kind(b, j, k < two, parity, b->stream));
    return LBM_OK;
}

int ensure_graph(lbm_batch *b, int steps) {
    if (b->graph && b->graph_steps == steps && b->graph_tiles2 == b->kind_tiles2) return LBM_OK;
    drop_graph(b);
    // One chain of launches on the batch's stream.  (Capturing one chain per kind on side
    // streams, so that the graph had independent branches, was dropped: replacing such a graph
    // between replays was followed by a host segmentation fault inside lbm_batch_step.)
    hipGraph_t g = nullptr;
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_steps(b, steps);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return bfail(b, LBM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    b->graph_steps = steps;
    b->graph_tiles2 = b->kind_tiles2;
    return LBM_OK;
}

bool any_active(const lbm_batch *b) {
    for (int i = 0; i < b->count; ++i)
        if (b->active[i]) return true;
    return false;
}

}  // namespace

extern "C" {

int lbm_batch_create(int count, const int *nx, const int *ny, const lbm_eos *eos,
                     const lbm_force *force, const lbm_collision *coll, const double *tau,
                     lbm_batch_t **out) {
    if (!out || count < 1 || !nx || !ny || !eos || !force || !coll || !tau) return LBM_EINVAL;
    *out = nullptr;
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ENOMEM;
    b->count = count;
    b->phys.resize(count);
    b->eos.assign(eos, eos + count);
    b->force.assign(force, force + count);
    for (int i = 0; i < count; ++i) {
        std::string why;
        int rc = pplbm::make_physics(nx[i], ny[i], &eos[i], &force[i], &coll[i], tau[i], &b->phys[i],
                                     nullptr, &why);
        if (!rc && pplbm::pop_bytes(b->phys[i]) > pplbm::kSweepMaxBytes) rc = LBM_EINVAL;
        if (rc) {
            delete b;
            return rc;
        }
    }
    for (int i = 0; i < count; ++i) b->kinds.push_back(pplbm::kernel_kind(b->phys[i].scheme));
    std::sort(b->kinds.begin(), b->kinds.end());
    b->kinds.erase(std::unique(b->kinds.begin(), b->kinds.end()), b->kinds.end());
    b->f0.assign(count, nullptr);
    b->f1.assign(count, nullptr);
    b->vprev.assign(count, nullptr);
    b->seg_rows.assign(count, 0);  // automatic
    b->active.assign(count, 0);
    b->initialised.assign(count, 0);
    b->steps.assign(count, 0);
    b->vprev_valid.assign(count, 0);
    b->xa.resize(count);
    b->ya.resize(count);
    b->xb.assign(count, 0);
    b->yb.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        b->xa[i] = nx[i] / 2;
        b->ya[i] = ny[i] / 2;
    }
    bool ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < count; ++i) {
        const Physics &p = b->phys[i];
        const size_t fb = 9 * p.plane * sizeof(float), vb = 2 * (size_t)p.nx * p.ny * sizeof(float);
        ok = hipMalloc(&b->f0[i], fb) == hipSuccess && hipMalloc(&b->f1[i], fb) == hipSuccess &&
             hipMalloc(&b->vprev[i], vb) == hipSuccess;
        ok = ok && hipMemsetAsync(b->f0[i], 0, fb, b->stream) == hipSuccess &&
             hipMemsetAsync(b->f1[i], 0, fb, b->stream) == hipSuccess;
    }
    ok = ok && hipMalloc(&b->desc, pplbm::batch_lattice_bytes() * count) == hipSuccess &&
         hipMalloc(&b->meta, 8 * sizeof(int2)) == hipSuccess &&
         hipMalloc(&b->meta2, 8 * sizeof(int2)) == hipSuccess &&
         hipMalloc(&b->out, pplbm::kStatsOut * sizeof(double) * count) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        lbm_batch_destroy(b);
        return LBM_ENOMEM;
    }
    if (upload_desc(b) || upload_tiles(b)) {
        lbm_batch_destroy(b);
        return LBM_EHIP;
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch_t *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (int i = 0; i < b->count; ++i) {
        if (b->f0[i]) (void)hipFree(b->f0[i]);
        if (b->f1[i]) (void)hipFree(b->f1[i]);
        if (b->vprev[i]) (void)hipFree(b->vprev[i]);
    }
    for (void *p : {(void *)b->desc, (void *)b->tiles, (void *)b->meta, (void *)b->tiles2,
                    (void *)b->meta2, (void *)b->sblocks,
                    (void *)b->ranges, (void *)b->ids, (void *)b->partial, (void *)b->out})
        if (p) (void)hipFree(p);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int lbm_batch_set_launch(lbm_batch_t *b, int tx, int groups, int flags) {
    if (!b) return LBM_EINVAL;
    if (tx < 64 || tx % 64 || tx > 512 || groups < 0)
        return bfail(b, LBM_EINVAL, "tx: multiple of 64 up to 512; groups >= 0 (0 = automatic)");
    if (flags & ~(LBM_LAUNCH_NONTEMPORAL | LBM_LAUNCH_SHALLOW | LBM_LAUNCH_SERIAL_KINDS |
                  LBM_LAUNCH_TWO_STEP))
        return bfail(b, LBM_EINVAL, "batch flags: LBM_LAUNCH_NONTEMPORAL, LBM_LAUNCH_SHALLOW, "
                                    "LBM_LAUNCH_SERIAL_KINDS, LBM_LAUNCH_TWO_STEP");
    drop_graph(b);
    b->tx = tx;
    b->groups = groups;
    b->flags = flags;
    int rc = upload_desc(b);
    return rc ? rc : upload_tiles(b);
}

int lbm_batch_set_segment(lbm_batch_t *b, int i, int rows) {
    if (!b || i < 0 || i >= b->count || rows < 0) return LBM_EINVAL;
    b->seg_rows[i] = rows;
    return upload_tiles(b);
}

int lbm_batch_set_active(lbm_batch_t *b, int i, int active) {
    if (!b || i < 0 || i >= b->count) return LBM_EINVAL;
    if (active && !b->initialised[i]) return bfail(b, LBM_ESTATE, "lattice not initialised");
    b->active[i] = active != 0;
    return upload_tiles(b);
}

int lbm_batch_init(lbm_batch_t *b, int i, const double *rho0, const double *u0) {
    if (!b || i < 0 || i >= b->count || !rho0) return LBM_EINVAL;
    const Physics &p = b->phys[i];
    const size_t N = (size_t)p.nx * p.ny;
    for (size_t k = 0; k < N; ++k)
        if (!(rho0[k] > 0) || (p.psi_kind == 0 && !(p.b_quarter * rho0[k] < 1)))
            return bfail(b, LBM_EUNSTABLE, "initial density outside (0, 4/b)");
    double *d = nullptr;
    if (hipMalloc(&d, N * sizeof(double) * (u0 ? 3 : 1)) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, LBM_ENOMEM, "staging allocation failed");
    }
    hipError_t e = hipMemcpyAsync(d, rho0, N * sizeof(double), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && u0)
        e = hipMemcpyAsync(d + N, u0, 2 * N * sizeof(double), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = pplbm::launch_init(p, d, u0 ? d + N : nullptr, b->f0[i], b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("lbm_batch_init: ") + hipGetErrorString(e));
    b->initialised[i] = 1;
    b->active[i] = 1;
    b->steps[i] = 0;
    b->vprev_valid[i] = 0;
    return upload_tiles(b);
}

namespace {
// f0 of lattice i, holding f^eq(rho, 0), becomes the force-consistent rest state.
static int rest_state(lbm_batch *b, int i) {
    const Physics &p = b->phys[i];
    float *psi = nullptr;
    if (hipMalloc(&psi, p.plane * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, LBM_ENOMEM, "psi scratch allocation failed");
    }
    hipError_t e = pplbm::launch_rest(p, b->f0[i], psi, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(psi);
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("rest state: ") + hipGetErrorString(e));
    return LBM_OK;
}
}  // namespace

int lbm_batch_init_rest(lbm_batch_t *b, int i, const double *rho0) {
    int rc = lbm_batch_init(b, i, rho0, nullptr);
    if (rc) return rc;
    rc = rest_state(b, i);
    if (rc) b->initialised[i] = b->active[i] = 0;
    const int up = upload_tiles(b);  // drops the lattice again if the rest state failed
    return rc ? rc : up;
}

int lbm_batch_init_tanh(lbm_batch_t *b, int i, double R, double W, int droplet) {
    if (!b || i < 0 || i >= b->count || !(R > 0) || !(W > 0)) return LBM_EINVAL;
    double g = 0, l = 0;
    int rc = lbm_coexistence(&b->eos[i], &b->force[i], LBM_COEX_MAXWELL, 0.0, &g, &l);
    if (rc) return bfail(b, rc, "no coexistence densities for this lattice's EOS");
    const Physics &p = b->phys[i];
    const double in = droplet ? l : g, out = droplet ? g : l;
    std::vector<double> rho((size_t)p.nx * p.ny);
    for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
            const double dx = x - 0.5 * p.nx, dy = y - 0.5 * p.ny;
            const double r = std::sqrt(dx * dx + dy * dy);
            rho[(size_t)y * p.nx + x] = 0.5 * (in + out) - 0.5 * (in - out) * std::tanh(2 * (r - R) / W);
        }
    return lbm_batch_init_rest(b, i, rho.data());
}

int lbm_batch_init_profile(lbm_batch_t *b, int i, const double *log_rho, double r0, double dr,
                           double mass, double *shift_out) {
    if (!b || i < 0 || i >= b->count || !log_rho || !(dr > 0) || !std::isfinite(r0))
        return bfail(b, LBM_EINVAL, "lbm_batch_init_profile: bad argument");
    for (int k = 0; k < 64; ++k)
        if (!std::isfinite(log_rho[k])) return bfail(b, LBM_EINVAL, "non-finite profile value");
    const Physics &p = b->phys[i];
    const int nb = pplbm::profile_mass_blocks(p);
    double *part = nullptr;
    if (hipMalloc(&part, 3 * (size_t)nb * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, LBM_ENOMEM, "staging allocation failed");
    }
    std::vector<double> host(3 * (size_t)nb);
    double lo_rho = 0, hi_rho = 0;
    // total mass, min and max density of the profile at a shift (partials added in order)
    auto measure = [&](double shift, double *sum) -> hipError_t {
        hipError_t e = pplbm::launch_profile_mass(p, log_rho, r0, dr, shift, part, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(host.data(), part, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                               b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return e;
        double s = 0, lo = INFINITY, hi = -INFINITY;
        for (int k = 0; k < nb; ++k) {
            s += host[3 * k];
            lo = std::fmin(lo, host[3 * k + 1]);
            hi = std::fmax(hi, host[3 * k + 2]);
        }
        *sum = s;
        lo_rho = lo;
        hi_rho = hi;
        return hipSuccess;
    };
    double shift = 0.0, m = 0;
    hipError_t e = hipSuccess;
    int rc = LBM_OK;
    if (mass > 0) {
        // the total mass is monotone in the shift (outwards: more of the inner phase); bisection
        // over shifts that move the profile by up to the lattice's half diagonal
        const double span = 0.5 * std::sqrt((double)p.nx * p.nx + (double)p.ny * p.ny);
        double lo = -span, hi = span, f_lo = 0, f_hi = 0;
        e = measure(lo, &f_lo);
        if (e == hipSuccess) e = measure(hi, &f_hi);
        f_lo -= mass;
        f_hi -= mass;
        if (e == hipSuccess && !((f_lo < 0 && f_hi > 0) || (f_lo > 0 && f_hi < 0))) {
            rc = bfail(b, LBM_EINVAL, "no shift of the profile carries that mass");
        } else {
            for (int it = 0; e == hipSuccess && it < 200; ++it) {
                shift = 0.5 * (lo + hi);
                e = measure(shift, &m);
                if (e != hipSuccess) break;
                const double d = m - mass;
                if (std::fabs(d) <= 1e-13 * mass) break;
                if ((d < 0) == (f_lo < 0)) {
                    lo = shift;
                    f_lo = d;
                } else {
                    hi = shift;
                }
            }
        }
    }
    if (e == hipSuccess && rc == LBM_OK) e = measure(shift, &m);
    if (e == hipSuccess && rc == LBM_OK && !(lo_rho > 0 && (p.psi_kind != 0 || p.b_quarter * hi_rho < 1)))
        rc = bfail(b, LBM_EUNSTABLE, "profile density outside (0, 4/b)");
    if (e == hipSuccess && rc == LBM_OK)
        e = pplbm::launch_profile_init(p, log_rho, r0, dr, shift, b->f0[i], b->stream);
    if (e == hipSuccess && rc == LBM_OK) e = hipStreamSynchronize(b->stream);
    (void)hipFree(part);
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("lbm_batch_init_profile: ") + hipGetErrorString(e));
    if (rc) return rc;
    rc = rest_state(b, i);
    if (rc) return rc;
    if (shift_out) *shift_out = shift;
    b->initialised[i] = 1;
    b->active[i] = 1;
    b->steps[i] = 0;
    b->vprev_valid[i] = 0;
    return upload_tiles(b);
}

namespace {
static int size_class(const Physics &p) {  // ceil(log2(longer side))
    int c = 0;
    while ((1 << c) < std::max(p.nx, p.ny)) ++c;
    return c;
}
}  // namespace

int lbm_batch_autotune(lbm_batch_t *b, const char *cache_path, int trial_steps, double *ms_out) {
    if (!b || trial_steps < 2 || trial_steps % 2) return bfail(b, LBM_EINVAL, "trial_steps: even, >= 2");
    for (int i = 0; i < b->count; ++i)
        if (!b->initialised[i]) return bfail(b, LBM_ESTATE, "lbm_batch_autotune before every lattice is initialised");
    // key: device and the multiset of (size, scheme, collision)
    std::vector<std::string> sig;
    for (int i = 0; i < b->count; ++i) {
        const Physics &p = b->phys[i];
        sig.push_back(std::to_string(p.nx) + "x" + std::to_string(p.ny) + "s" + std::to_string(p.scheme) + "c" +
                      std::to_string(p.coll));
    }
    std::sort(sig.begin(), sig.end());
    unsigned long long hsh = 1469598103934665603ull;  // FNV-1a
    for (const std::string &t : sig)
        for (char c : t + ";") hsh = (hsh ^ (unsigned char)c) * 1099511628211ull;
    std::vector<int> classes;
    for (int i = 0; i < b->count; ++i) classes.push_back(size_class(b->phys[i]));
    std::vector<int> distinct = classes;
    std::sort(distinct.begin(), distinct.end());
    distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
    char hex[24];
    std::snprintf(hex, sizeof hex, "%016llx", hsh);
    const std::string key = pplbm::device_tag() + "|batch|" + std::to_string(b->count) + "|" + hex;

    auto apply = [&](int tx, int fl, const std::vector<int> &rows_of_class) -> int {
        for (int i = 0; i < b->count; ++i) {
            const size_t c = std::lower_bound(distinct.begin(), distinct.end(), classes[i]) - distinct.begin();
            b->seg_rows[i] = rows_of_class[c];
        }
        return lbm_batch_set_launch(b, tx, b->groups, fl);
    };
    std::string hit;
    if (pplbm::tune_cache_lookup(cache_path, key, &hit)) {
        std::istringstream in(hit);
        int tx = 0, fl = 0;
        std::vector<int> rows(distinct.size(), 32);
        bool ok = static_cast<bool>(in >> tx >> fl);
        for (size_t c = 0; ok && c < distinct.size(); ++c) ok = static_cast<bool>(in >> rows[c]) && rows[c] >= 0;
        if (ok && apply(tx, fl, rows) == LBM_OK) {
            if (ms_out) *ms_out = -1.0;
            return LBM_OK;
        }
    }
    // save the current populations (every lattice sits at an even step, so in f0)
    std::vector<float *> saved(b->count, nullptr);
    int rc = LBM_OK;
    for (int i = 0; i < b->count && !rc; ++i) {
        const size_t fb = 9 * b->phys[i].plane * sizeof(float);
        if (hipMalloc(&saved[i], fb) != hipSuccess) {
            (void)hipGetLastError();
            saved[i] = nullptr;
            rc = bfail(b, LBM_ENOMEM, "autotune: state copy allocation failed");
        } else if (hipMemcpyAsync(saved[i], b->f0[i], fb, hipMemcpyDeviceToDevice, b->stream) != hipSuccess) {
            rc = bfail(b, LBM_EHIP, "autotune: state copy failed");
        }
    }
    const std::vector<long long> steps0 = b->steps;
    const std::vector<char> active0 = b->active;
    const int tx0 = b->tx, fl0 = b->flags;
    std::vector<int> rows0(distinct.size(), 32);
    for (int i = 0; i < b->count; ++i)
        rows0[std::lower_bound(distinct.begin(), distinct.end(), classes[i]) - distinct.begin()] = b->seg_rows[i];
    for (int i = 0; i < b->count; ++i) b->active[i] = 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = bfail(b, LBM_EHIP, "autotune: event creation failed");
    auto trial = [&](int tx, int fl, const std::vector<int> &rows, double *ms) -> int {
        int r = apply(tx, fl, rows);
        if (!r) r = lbm_batch_step(b, 2);
        if (r) return r;
        BHIP(b, hipEventRecord(e0, b->stream));
        r = lbm_batch_step(b, trial_steps);
        if (r) return r;
        BHIP(b, hipEventRecord(e1, b->stream));
        BHIP(b, hipEventSynchronize(e1));
        float t = 0;
        BHIP(b, hipEventElapsedTime(&t, e0, e1));
        *ms = t / trial_steps;
        return LBM_OK;
    };
    int best_tx = tx0, best_fl = fl0;
    std::vector<int> best_rows = rows0;
    double best_ms = 1e300, ms = 0;
    // stage 1: strip width and prefetch depth at the current segment heights
    for (int tx : {64, 128, 256, 512}) {
        for (int fl : {pplbm::kFlagShallow, 0, (int)LBM_LAUNCH_TWO_STEP}) {
            if (rc) break;
            rc = trial(tx, fl, rows0, &ms);
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best_tx = tx;
                best_fl = fl;
            }
        }
    }
    // stage 2: segment height per size class, one class at a time
    for (size_t c = 0; c < distinct.size() && !rc; ++c) {
        for (int rows : {8, 16, 32, 64}) {
            if (rc) break;
            std::vector<int> cand = best_rows;
            cand[c] = rows;
            rc = trial(best_tx, best_fl, cand, &ms);
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best_rows = cand;
            }
        }
    }
    // restore the state and the activity flags whatever happened
    for (int i = 0; i < b->count; ++i) {
        if (saved[i]) {
            if (hipMemcpyAsync(b->f0[i], saved[i], 9 * b->phys[i].plane * sizeof(float), hipMemcpyDeviceToDevice,
                               b->stream) != hipSuccess && !rc)
                rc = bfail(b, LBM_EHIP, "autotune: state restore failed");
        }
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess && !rc) rc = bfail(b, LBM_EHIP, "autotune: sync failed");
    for (float *q : saved)
        if (q) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->steps = steps0;
    b->active = active0;
    const int rc2 = rc ? apply(tx0, fl0, rows0) : apply(best_tx, best_fl, best_rows);
    if (rc) return rc;
    if (rc2) return rc2;
    std::ostringstream val;
    val << best_tx << " " << best_fl;
    for (int r : best_rows) val << " " << r;
    pplbm::tune_cache_store(cache_path, key, val.str(), best_ms);
    if (ms_out) *ms_out = best_ms;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch_t *b, int n) {
    if (!b || n < 0 || n % 2) return bfail(b, LBM_EINVAL, "lbm_batch_step: n must be even and >= 0");
    if (b->tiles_dirty) {
        int rc = upload_tiles(b);
        if (rc) return rc;
    }
    if (!n || !any_active(b)) return LBM_OK;
    int rc = ensure_graph(b, n);
    if (rc) return rc;
    BHIP(b, hipGraphLaunch(b->graph, b->stream));
    for (int i = 0; i < b->count; ++i)
        if (b->active[i]) b->steps[i] += n;
    return LBM_OK;
}

// FP64 observables of every active lattice (out[i] for active i; others untouched).
int lbm_batch_stats(lbm_batch_t *b, int track_dv, lbm_stats_t *out) {
    if (!b || !out) return LBM_EINVAL;
    std::vector<int4> sb;
    std::vector<int2> ranges;
    std::vector<int> ids;
    for (int i = 0; i < b->count; ++i) {
        if (!b->active[i]) continue;
        const Physics &p = b->phys[i];
        const size_t N = (size_t)p.nx * p.ny;
        const int chunks = (int)std::min<size_t>((N + 255) / 256, 64);
        ranges.push_back(make_int2((int)sb.size(), chunks));
        ids.push_back(i);
        for (int c = 0; c < chunks; ++c) sb.push_back(make_int4(i, c, chunks, (int)sb.size()));
    }
    if (ids.empty()) return LBM_OK;
    if (sb.size() > b->max_sblocks) {
        for (void *p : {(void *)b->sblocks, (void *)b->ranges, (void *)b->ids, (void *)b->partial})
            if (p) (void)hipFree(p);
        b->sblocks = nullptr;
        b->ranges = nullptr;
        b->ids = nullptr;
        b->partial = nullptr;
        const size_t m = sb.size();
        if (hipMalloc(&b->sblocks, m * sizeof(int4)) != hipSuccess ||
            hipMalloc(&b->ranges, b->count * sizeof(int2)) != hipSuccess ||
            hipMalloc(&b->ids, b->count * sizeof(int)) != hipSuccess ||
            hipMalloc(&b->partial, m * pplbm::kStatsFields * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            b->max_sblocks = 0;
            return bfail(b, LBM_ENOMEM, "reduction buffers");
        }
        b->max_sblocks = m;
    }
    BHIP(b, hipMemcpyAsync(b->sblocks, sb.data(), sb.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->ranges, ranges.data(), ranges.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->ids, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
    BHIP(b, pplbm::launch_batch_stats(b->desc, b->sblocks, (int)sb.size(), b->ranges, b->ids,
                                      (int)ids.size(), 0, track_dv, b->partial, b->out, b->stream));
    std::vector<double> r(pplbm::kStatsOut * b->count);
    BHIP(b, hipMemcpyAsync(r.data(), b->out, r.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    int unstable = 0;
    for (int i : ids) {
        const double *q = &r[(size_t)i * pplbm::kStatsOut];
        lbm_stats_t &s = out[i];
        s.mass = q[0];
        s.rho_min = q[1];
        s.rho_max = q[2];
        s.us_max = q[3];
        s.dv_max = (track_dv && b->vprev_valid[i]) ? q[4] : 0.0;
        s.nonfinite = (int)q[5];
        s.rho_probe_a = q[6];
        s.rho_probe_b = q[7];
        s.ratio = std::fmax(q[6], q[7]) / std::fmin(q[6], q[7]);
        s.step = b->steps[i];
        if (track_dv) b->vprev_valid[i] = 1;
        if (s.nonfinite) unstable = 1;
    }
    return unstable ? LBM_EUNSTABLE : LBM_OK;
}

int lbm_batch_run(lbm_batch_t *b, double tol, double tol_rho, int check_every,
                  long long max_steps, long long *steps_out, int *status_out) {
    if (!b || !(tol > 0) || check_every < 2 || check_every % 2 || max_steps < 0)
        return bfail(b, LBM_EINVAL, "lbm_batch_run: tol > 0, even check_every >= 2");
    std::vector<lbm_stats_t> st(b->count);
    std::vector<double> pa(b->count, 0.0), pb(b->count, 0.0);
    for (int i = 0; i < b->count; ++i)
        if (status_out) status_out[i] = b->active[i] ? LBM_ENOTCONVERGED : LBM_ESTATE;
    int rc = lbm_batch_stats(b, 1, st.data());  // first velocity snapshot
    if (rc && rc != LBM_EUNSTABLE) return rc;
    for (int i = 0; i < b->count; ++i) {
        pa[i] = st[i].rho_probe_a;
        pb[i] = st[i].rho_probe_b;
    }
    while (any_active(b)) {
        rc = lbm_batch_step(b, check_every);
        if (rc) return rc;
        rc = lbm_batch_stats(b, 1, st.data());
        if (rc && rc != LBM_EUNSTABLE) return rc;
        bool changed = false;
        for (int i = 0; i < b->count; ++i) {
            if (!b->active[i]) continue;
            // per-step relative change of the two probe densities over the check interval
            const double dr = std::fmax(std::fabs(st[i].rho_probe_a - pa[i]) / st[i].rho_probe_a,
                                        std::fabs(st[i].rho_probe_b - pb[i]) / st[i].rho_probe_b) /
                              check_every;
            pa[i] = st[i].rho_probe_a;
            pb[i] = st[i].rho_probe_b;
            int status = 1;  // still running
            if (st[i].nonfinite) status = LBM_EUNSTABLE;
            else if (st[i].dv_max / check_every < tol && (!(tol_rho > 0) || dr < tol_rho)) status = LBM_OK;
            else if (b->steps[i] >= max_steps) status = LBM_ENOTCONVERGED;
            if (status != 1) {
                b->active[i] = 0;
                changed = true;
                if (status_out) status_out[i] = status;
            }
        }
        if (changed) {
            rc = upload_tiles(b);
            if (rc) return rc;
        }
    }
    if (steps_out)
        for (int i = 0; i < b->count; ++i) steps_out[i] = b->steps[i];
    return LBM_OK;
}

int lbm_batch_read(lbm_batch_t *b, int i, double *rho, double *u) {
    if (!b || i < 0 || i >= b->count) return LBM_EINVAL;
    if (!b->initialised[i]) return bfail(b, LBM_ESTATE, "lattice not initialised");
    const Physics &p = b->phys[i];
    const size_t N = (size_t)p.nx * p.ny;
    double *d = nullptr;
    float *psi = nullptr;
    if (hipMalloc(&d, 3 * N * sizeof(double)) != hipSuccess || hipMalloc(&psi, p.plane * sizeof(float)) != hipSuccess) {
        if (d) (void)hipFree(d);
        (void)hipGetLastError();
        return bfail(b, LBM_ENOMEM, "staging allocation failed");
    }
    hipError_t e = pplbm::launch_psi(p, pplbm::kPrecF64, 0, b->f0[i], psi, b->stream);
    if (e == hipSuccess) e = pplbm::launch_macro(p, b->f0[i], psi, d, d + N, b->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, N * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, d + N, 2 * N * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    (void)hipFree(psi);
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("lbm_batch_read: ") + hipGetErrorString(e));
    return LBM_OK;
}

int lbm_batch_populations(lbm_batch_t *b, int i, float *f) {
    if (!b || i < 0 || i >= b->count || !f) return LBM_EINVAL;
    const Physics &p = b->phys[i];
    for (int q = 0; q < 9; ++q)
        BHIP(b, hipMemcpy2DAsync(f + (size_t)q * p.nx * p.ny, p.nx * sizeof(float), b->f0[i] + q * p.fq,
                                 p.frow * sizeof(float), p.nx * sizeof(float), p.ny, hipMemcpyDeviceToHost,
                                 b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

long long lbm_batch_steps(const lbm_batch_t *b, int i) {
    if (!b || i < 0 || i >= b->count) return -1;
    return b->steps[i];
}

int lbm_batch_sync(lbm_batch_t *b) {
    if (!b) return LBM_EINVAL;
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch_t *b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
