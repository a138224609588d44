// Drives the library's host-only code paths, for a build whose host code carries the address
// and undefined-behaviour sanitizers: parameter validation of lbm_create and
// lbm_batch_create, the launch rules, the EOS helpers (critical point, Maxwell densities,
// bulk pressure), the flat-interface coexistence solver of both rules and both psi kinds, the
// checkpoint reader on foreign and truncated files, and the autotuner cache parser on
// malformed lines.  Nothing here touches a GPU.  Exit status 0 when every call returned what
// it should.
#include <cmath>
#include <cstdio>
#include <string>

#include "pplbm.h"

namespace pplbm {
bool tune_cache_lookup(const char *path, const std::string &key, std::string *value);
bool tune_cache_store(const char *path, const std::string &key, const std::string &value, double ms);
}  // namespace pplbm

static int failures = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

int main(int argc, char **argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    lbm_eos eos{LBM_EOS_CARNAHAN_STARLING, 1.0, 4.0, 1.0, 0.6, 1.0 / 49, 0.0};
    lbm_force frc{LBM_FORCE_GUO_LI, 0.0, 0.125, -1.0};
    lbm_collision col{LBM_COLL_MRT, 1.0, 1.1, 1.1, 1.0, 1.1};
    // validation
    lbm_t *h = nullptr;
    CHECK(lbm_create(0, 5, &eos, &frc, &col, 1.0, &h) == LBM_EINVAL && !h);
    CHECK(lbm_create(5, 5, &eos, &frc, &col, 0.5, &h) == LBM_EINVAL);
    lbm_force edm{LBM_FORCE_EDM, -0.26, 0.0, -1.0};
    CHECK(lbm_create(5, 5, &eos, &edm, &col, 1.0, &h) == LBM_EINVAL);
    CHECK(lbm_create(5, 5, &eos, nullptr, &col, 1.0, &h) == LBM_EINVAL);
    for (int nx : {1, 3, 57, 58, 59, 4096})
        for (int ny : {1, 5, 64, 4096}) {
            CHECK(lbm_create(nx, ny, &eos, &frc, &col, 1.0, &h) == LBM_OK && h);
            int k = -1, tx = 0, ty = 0, fl = 0;
            CHECK(lbm_get_launch(h, &k, &tx, &ty, &fl) == LBM_OK && k == LBM_KERNEL_SWEEP2 && ty >= 1 &&
                  (ty >= 6 || tx == 64));
            CHECK(lbm_set_launch(h, LBM_KERNEL_SWEEP, 512, 8, LBM_LAUNCH_XCD_ORDER) == LBM_OK);
            CHECK(lbm_set_launch(h, LBM_KERNEL_SWEEP2, 320, 8, 0) == LBM_EINVAL);
            CHECK(lbm_set_precision(h, 0) == LBM_EINVAL && lbm_set_precision(h, LBM_PREC_F64) == 0);
            CHECK(lbm_set_probes(h, nx, 0, 0, 0) == LBM_EINVAL);
            CHECK(lbm_step(h, 1) == LBM_ESTATE);
            lbm_stats_t st;
            CHECK(lbm_stats(h, 0, &st) == LBM_ESTATE && lbm_stats_noalloc(h, &st) == LBM_ESTATE);
            CHECK(lbm_load(h, (dir + "/missing.ckpt").c_str()) == LBM_EINVAL);
            lbm_destroy(h);
            h = nullptr;
        }
    // checkpoint reader: a foreign file and a truncated header
    {
        const std::string p1 = dir + "/foreign.ckpt", p2 = dir + "/short.ckpt";
        FILE *fp = std::fopen(p1.c_str(), "wb");
        std::fputs("not a checkpoint of anything at all, but long enough to read a header", fp);
        std::fclose(fp);
        fp = std::fopen(p2.c_str(), "wb");
        std::fwrite("PPLBMCK1\x05\x00", 1, 10, fp);
        std::fclose(fp);
        CHECK(lbm_create(5, 5, &eos, &frc, &col, 1.0, &h) == LBM_OK);
        CHECK(lbm_load(h, p1.c_str()) == LBM_EINVAL);
        CHECK(lbm_load(h, p2.c_str()) == LBM_EINVAL);
        lbm_destroy(h);
    }
    // batch validation
    {
        int nx[2] = {64, 0}, ny[2] = {64, 64};
        lbm_eos e2[2] = {eos, eos};
        lbm_force f2[2] = {frc, frc};
        lbm_collision c2[2] = {col, col};
        double tau[2] = {1.0, 1.0};
        lbm_batch_t *b = nullptr;
        CHECK(lbm_batch_create(2, nx, ny, e2, f2, c2, tau, &b) == LBM_EINVAL && !b);
        CHECK(lbm_batch_create(0, nx, ny, e2, f2, c2, tau, &b) == LBM_EINVAL);
    }
    // EOS helpers and the coexistence solver
    double rc = 0, Tc = 0, pc = 0, g = 0, l = 0, p = 0;
    CHECK(lbm_eos_critical(&eos, &rc, &Tc, &pc) == LBM_OK && std::fabs(Tc - 0.0943287031) < 1e-9);
    for (double t : {0.3, 0.5, 0.6, 0.8, 0.9, 0.99}) {
        lbm_eos e = eos;
        e.T_over_Tc = t;
        CHECK(lbm_eos_maxwell(&e, &g, &l) == LBM_OK && g > 0 && g < l);
        CHECK(lbm_coexistence(&e, &frc, LBM_COEX_MAXWELL, 0.0, &g, &l) == LBM_OK);
        const int rm = lbm_coexistence(&e, &frc, LBM_COEX_MECHANICAL, 2.0, &g, &l);
        CHECK(rm == LBM_OK || rm == LBM_EINVAL);
        CHECK(lbm_eos_pressure(&e, &frc, 0.2, &p) == LBM_OK && std::isfinite(p));
    }
    lbm_eos hot = eos;
    hot.T_over_Tc = 1.2;
    CHECK(lbm_eos_maxwell(&hot, &g, &l) == LBM_EINVAL);
    CHECK(lbm_coexistence(&hot, &frc, LBM_COEX_MAXWELL, 0.0, &g, &l) == LBM_EINVAL);
    for (double eps : {0.0, 1.0}) {
        lbm_eos ss{LBM_EOS_SBRAGAGLIA_SHAN, 1.0, 4.0, 1.0, 0.5, 1.0, eps};
        lbm_force fs{LBM_FORCE_GUO, -eps / 2, 0.0, eps ? -3.0 : -4.0};
        CHECK(lbm_coexistence(&ss, &fs, LBM_COEX_MAXWELL, 0.0, &g, &l) == LBM_OK);
        CHECK(lbm_coexistence(&ss, &fs, LBM_COEX_MECHANICAL, eps, &g, &l) == LBM_OK);
    }
    // autotuner cache: malformed lines are skipped, a store replaces its key's line
    {
        const std::string path = dir + "/tune.jsonl";
        FILE *fp = std::fopen(path.c_str(), "w");
        std::fputs("{\"key\": \"a|b\", \"value\": \"1 2 3 4\", \"ms\": 0.5}\n"
                   "{\"key\": \"broken\n\"value\": \"9\"}\n{\"key\"\n\n{}\n", fp);
        std::fclose(fp);
        std::string v;
        CHECK(pplbm::tune_cache_lookup(path.c_str(), "a|b", &v) && v == "1 2 3 4");
        CHECK(!pplbm::tune_cache_lookup(path.c_str(), "missing", &v));
        CHECK(!pplbm::tune_cache_lookup(nullptr, "a|b", &v));
        CHECK(pplbm::tune_cache_store(path.c_str(), "a|b", "5 6 7 8", 0.25));
        CHECK(pplbm::tune_cache_lookup(path.c_str(), "a|b", &v) && v == "5 6 7 8");
        CHECK(!pplbm::tune_cache_lookup((dir + "/no_such_file").c_str(), "a|b", &v));
    }
    std::printf("%s\n", lbm_strerror(LBM_EUNSTABLE));
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::puts("host driver: ok");
    return 0;
}
