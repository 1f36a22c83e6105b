// Drives the host code of the library (symbolic analysis) and the C oracle on
// seeded random patterns and systems, for an AddressSanitizer /
// UndefinedBehaviorSanitizer build on the CPU (tests/test_sanitize.py builds
// and runs it). Exit status 0 = every call returned what it should and the
// sanitizers reported nothing.
#include "../../paper_2110_03636_amd/csrc/analysis.hpp"

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
typedef struct orc orc;
typedef struct {
    double cg_tol, kkt_tol, qf_eps, delta2;
    int64_t max_cg, max_refine, inexact;
} orc_opts;
typedef struct {
    int64_t status, passes, cg_iters[16];
    double rr_hist[16], rr, be, floor;
    int64_t inertia[3];
} orc_report;
orc* orc_new(int64_t n, int64_t m, const int64_t* Hp, const int32_t* Hi, const double* Hx, const double* Dx,
             const int64_t* Jp, const int32_t* Ji, const double* Jx, double delta, double gamma);
void orc_free(orc* s);
void orc_order_mindeg(const orc* s, int32_t* perm);
int orc_factor(orc* s, const int32_t* perm, int64_t* fail_col);
int orc_solve(orc* s, const orc_opts* o, const double* r1, const double* r2, double* x, double* y, orc_report* rep);
void orc_ruiz(const orc* s, int64_t iters, double* d);
int orc_solve_scaled(orc* s, const orc_opts* o, const double* d, const int32_t* perm, const double* r1,
                     const double* r2, double* x, double* y, orc_report* rep);
int orc_factor_regularized(orc* s, const int32_t* perm, double* delta_min, double delta_max, double* delta1,
                           int64_t* fail_col);
int64_t orc_refine_dd(orc* s, const orc_opts* o, const double* r1, const double* r2, double* x, double* y,
                      int64_t max_steps, double* hist);
void orc_metrics(orc* s, const double* r1, const double* r2, const double* x, const double* y, double* out3);
typedef struct orc4 orc4;
orc4* orc4_new(int64_t n, int64_t m, int64_t md, const int64_t* Hp, const int32_t* Hi, const double* Hx,
               const double* Dx, const int64_t* Jp, const int32_t* Ji, const double* Jx, const int64_t* Dp,
               const int32_t* Di, const double* Dv, const double* Ds, double delta, double gamma);
void orc4_free(orc4* q);
orc* orc4_two(orc4* q);
void orc4_solve(orc4* q, const orc_opts* o, const double* rx, const double* rs, const double* ry, const double* ryd,
                double* x, double* sv, double* y, double* yd, double* out);
}

static uint64_t rng_state = 12345;
static uint64_t next_u64() {   // splitmix64
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double uni() { return (double)(next_u64() >> 11) * 0x1.0p-53; }
static int below(int k) { return (int)(next_u64() % (uint64_t)k); }

struct Pat {
    int64_t n, m;
    std::vector<int64_t> Hp, Jp;
    std::vector<int32_t> Hi, Ji;
};

// tril(H): diagonal plus a few neighbours within a band; J: m rows, a unit-like
// column plus three more, sorted and unique
static Pat make(int64_t n, int64_t m, int band) {
    Pat p;
    p.n = n;
    p.m = m;
    p.Hp.push_back(0);
    for (int64_t i = 0; i < n; i++) {
        std::vector<int32_t> r{(int32_t)i};
        for (int k = 0; k < 2 && i > 0; k++) r.push_back((int32_t)std::max<int64_t>(0, i - 1 - below(band)));
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        p.Hi.insert(p.Hi.end(), r.begin(), r.end());
        p.Hp.push_back((int64_t)p.Hi.size());
    }
    p.Jp.push_back(0);
    for (int64_t r = 0; r < m; r++) {
        std::vector<int32_t> c{(int32_t)((2 * r) % n)};
        for (int k = 0; k < 3; k++) c.push_back(below((int)n));
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        p.Ji.insert(p.Ji.end(), c.begin(), c.end());
        p.Jp.push_back((int64_t)p.Ji.size());
    }
    return p;
}

static int fails = 0;
#define CHECK(cond, ...)                       \
    do {                                       \
        if (!(cond)) {                         \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");        \
            fails++;                           \
        }                                      \
    } while (0)

static void run_analysis() {
    for (int64_t n : {1, 7, 130, 900, 3000})
        for (int ordering : {0, 1, 2})
            for (int relax : {0, 1, 2}) {
                Pat p = make(n, n / 2, 12);
                hkkt::Symbolic S;
                hkkt::AnalyzeOptions o;
                o.ordering = ordering;
                o.relax = relax;
                const std::string e = hkkt::analyze(S, p.n, p.m, p.Hp.data(), p.Hi.data(), p.Jp.data(), p.Ji.data(),
                                                    nullptr, o);
                CHECK(e.empty(), "analyze n=%lld ord=%d relax=%d: %s", (long long)n, ordering, relax, e.c_str());
            }
    // a group of three members as one block-diagonal pattern
    {
        std::vector<Pat> mem{make(300, 150, 8), make(90, 0, 4), make(500, 250, 16)};
        Pat g;
        g.n = g.m = 0;
        g.Hp.push_back(0);
        g.Jp.push_back(0);
        std::vector<int64_t> xo{0}, yo{0};
        for (const Pat& p : mem) {
            for (int64_t i = 0; i < p.n; i++) {
                for (int64_t q = p.Hp[i]; q < p.Hp[i + 1]; q++) g.Hi.push_back((int32_t)(p.Hi[q] + g.n));
                g.Hp.push_back((int64_t)g.Hi.size());
            }
            for (int64_t r = 0; r < p.m; r++) {
                for (int64_t q = p.Jp[r]; q < p.Jp[r + 1]; q++) g.Ji.push_back((int32_t)(p.Ji[q] + g.n));
                g.Jp.push_back((int64_t)g.Ji.size());
            }
            g.n += p.n;
            g.m += p.m;
            xo.push_back(g.n);
            yo.push_back(g.m);
        }
        for (int ordering : {0, 2}) {
            hkkt::Symbolic S;
            hkkt::AnalyzeOptions o;
            o.ordering = ordering;
            const std::string e = hkkt::analyze(S, g.n, g.m, g.Hp.data(), g.Hi.data(), g.Jp.data(), g.Ji.data(),
                                                nullptr, o, 3, xo.data(), yo.data());
            CHECK(e.empty(), "group analyze ord=%d: %s", ordering, e.c_str());
        }
    }
    // malformed patterns are rejected, not read out of bounds
    {
        Pat p = make(50, 20, 5);
        std::swap(p.Hi[p.Hp[10]], p.Hi[p.Hp[10] + 1]);   // unsorted row (rows there hold two entries or more)
        Pat q = make(50, 20, 5);
        q.Ji[3] = 50;                                      // column out of range
        for (Pat* bad : {&p, &q}) {
            hkkt::Symbolic S;
            hkkt::AnalyzeOptions o;
            const std::string e = hkkt::analyze(S, bad->n, bad->m, bad->Hp.data(), bad->Hi.data(), bad->Jp.data(),
                                                bad->Ji.data(), nullptr, o);
            CHECK(!e.empty(), "malformed pattern accepted");
        }
    }
}

static void run_oracle() {
    for (int64_t n : {12, 60, 400}) {
        const int64_t m = n / 3;
        Pat p = make(n, m, 6);
        std::vector<double> Hx(p.Hi.size()), Dx(n), Jx(p.Ji.size()), r1(n), r2(m), x(n), y(m);
        for (int64_t i = 0; i < n; i++)
            for (int64_t q = p.Hp[i]; q < p.Hp[i + 1]; q++) Hx[q] = p.Hi[q] == i ? 4.0 + uni() : -0.5 * uni();
        for (auto& v : Dx) v = 0.1 + uni();
        for (auto& v : Jx) v = uni() - 0.5;
        for (int64_t r = 0; r < m; r++) Jx[p.Jp[r]] += 2.0;   // a dominant entry per row
        for (auto& v : r1) v = uni() - 0.5;
        for (auto& v : r2) v = uni() - 0.5;
        orc* s = orc_new(n, m, p.Hp.data(), p.Hi.data(), Hx.data(), Dx.data(), p.Jp.data(), p.Ji.data(), Jx.data(),
                         1e-8, 1e2);
        std::vector<int32_t> perm(n);
        orc_order_mindeg(s, perm.data());
        int64_t fc = 0;
        CHECK(orc_factor(s, perm.data(), &fc) == 0, "oracle factor n=%lld", (long long)n);
        orc_opts o{1e-12, 1e-10, 1e-14, 0.0, 0, 10, 1};
        orc_report rep;
        orc_solve(s, &o, r1.data(), r2.data(), x.data(), y.data(), &rep);
        CHECK(rep.status == 0, "oracle solve n=%lld status %lld rr %g", (long long)n, (long long)rep.status, rep.rr);
        std::vector<double> d(n + m), hist(9);
        orc_ruiz(s, 10, d.data());
        orc_solve_scaled(s, &o, d.data(), perm.data(), r1.data(), r2.data(), x.data(), y.data(), &rep);
        CHECK(rep.status == 0, "oracle scaled solve n=%lld", (long long)n);
        orc_refine_dd(s, &o, r1.data(), r2.data(), x.data(), y.data(), 8, hist.data());
        double mt[3];
        orc_metrics(s, r1.data(), r2.data(), x.data(), y.data(), mt);
        double dmin = 1e-9, d1 = 0.0;
        orc_factor_regularized(s, perm.data(), &dmin, 1e-6, &d1, &fc);
        orc_free(s);
        // the 4x4 system
        const int64_t md = n / 4;
        std::vector<int64_t> Dp{0};
        std::vector<int32_t> Di;
        for (int64_t k = 0; k < md; k++) {
            std::vector<int32_t> c{(int32_t)below((int)n), (int32_t)below((int)n), (int32_t)below((int)n)};
            std::sort(c.begin(), c.end());
            c.erase(std::unique(c.begin(), c.end()), c.end());
            Di.insert(Di.end(), c.begin(), c.end());
            Dp.push_back((int64_t)Di.size());
        }
        std::vector<double> Dv(Di.size()), Ds(md), rs(md), ryd(md), sv(md), yd(md);
        for (auto& v : Dv) v = uni() - 0.5;
        for (auto& v : Ds) v = 0.5 + uni();
        for (auto& v : rs) v = uni() - 0.5;
        for (auto& v : ryd) v = uni() - 0.5;
        orc4* q = orc4_new(n, m, md, p.Hp.data(), p.Hi.data(), Hx.data(), Dx.data(), p.Jp.data(), p.Ji.data(),
                           Jx.data(), Dp.data(), Di.data(), Dv.data(), Ds.data(), 1e-8, 1e2);
        CHECK(orc_factor(orc4_two(q), nullptr, &fc) == 0, "oracle 4x4 factor");
        double out[5];
        orc4_solve(q, &o, r1.data(), rs.data(), r2.data(), ryd.data(), x.data(), sv.data(), y.data(), yd.data(), out);
        CHECK(out[4] == 0.0, "oracle 4x4 solve n=%lld rr %g", (long long)n, out[0]);
        orc4_free(q);
    }
}

int main() {
    run_analysis();
    run_oracle();
    std::printf("host driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
