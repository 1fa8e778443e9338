// Host-only checks of the dsx runtime under AddressSanitizer / UndefinedBehaviorSanitizer:
//   1. the serving arena (first-fit sub-allocation with coalescing) under a randomized
//      allocate / release sequence, against a shadow list of live ranges;
//   2. the host-only C-ABI calls (dsx_plan_query, dsx_split_sites) with valid and
//      invalid inputs, and with every heap allocation they make failing in turn
//      (operator new of this program fails after a set count): each call returns
//      DSX_OK or DSX_ERR_NOMEM, never crashes, and leaks nothing.
// No GPU is touched.  Exit status 0 on success; prints the failing check otherwise.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "arena.h"
#include "dsx.h"

static long g_fail_after = -1;   // < 0: never fail; else the number of allocations that succeed

void* operator new(std::size_t n)
{
    if (g_fail_after == 0) throw std::bad_alloc();
    if (g_fail_after > 0) --g_fail_after;
    void* p = std::malloc(n ? n : 1);
    if (!p) throw std::bad_alloc();
    return p;
}
void* operator new[](std::size_t n) { return operator new(n); }
void* operator new(std::size_t n, const std::nothrow_t&) noexcept
{
    try { return operator new(n); } catch (...) { return nullptr; }
}
void* operator new[](std::size_t n, const std::nothrow_t&) noexcept
{
    try { return operator new(n); } catch (...) { return nullptr; }
}
void operator delete(void* p) noexcept { std::free(p); }
void operator delete[](void* p) noexcept { std::free(p); }
void operator delete(void* p, std::size_t) noexcept { std::free(p); }
void operator delete[](void* p, std::size_t) noexcept { std::free(p); }

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

static void arena_stress()
{
    const size_t size = 1 << 24;
    dsx::Arena a;
    a.init(size);
    struct Live { size_t off, n; };
    std::vector<Live> live;
    std::mt19937_64 rng(12345);
    size_t used = 0;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t n = 1 + rng() % (size / 64);
            size_t off = 0;
            const bool ok = a.alloc(n, &off);
            if (ok) {
                const size_t r = dsx::Arena::round(n);
                CHECK(off % 256 == 0 && off + r <= size);
                for (const Live& l : live) CHECK(off + r <= l.off || l.off + l.n <= off);
                live.push_back({off, r});
                used += r;
            } else {
                CHECK(used + dsx::Arena::round(n) > size || live.size() > 1);
            }
        } else {
            const size_t i = rng() % live.size();
            a.release(live[i].off, live[i].n);
            used -= live[i].n;
            live.erase(live.begin() + (long)i);
        }
        CHECK(a.peak() <= size);
    }
    for (const Live& l : live) a.release(l.off, l.n);
    // everything coalesced back into one range
    size_t off = 1;
    CHECK(a.alloc(size, &off) && off == 0);
}

static dsx_model_desc fcc_desc(const double* frac, const double* b, int order)
{
    dsx_model_desc d;
    std::memset(&d, 0, sizeof(d));
    const double cell[6] = {4, 4, 4, 90, 90, 90};
    std::memcpy(d.cell, cell, sizeof(cell));
    d.n[0] = 8; d.n[1] = 6; d.n[2] = 5;
    d.n_sites = 4;
    d.frac = frac;
    d.b = b;
    d.kind = DSX_NUCLEAR;
    d.taylor_order = order;
    d.n_configs = 2;
    return d;
}

// Inputs and outputs of the split-site call, allocated before any allocation is made to
// fail (only the library's own allocations are failed).
struct SplitBuffers {
    static const int M = 2, S = 4, ncell = 24, maxs = 16;
    std::vector<float> disp = std::vector<float>((size_t)M * S * ncell * 3);
    std::vector<float> occ = std::vector<float>((size_t)M * S * ncell, 1.f);
    std::vector<double> fo = std::vector<double>(maxs * 3), bo = std::vector<double>(maxs);
    std::vector<int32_t> po = std::vector<int32_t>(maxs);
    std::vector<float> oo = std::vector<float>((size_t)M * maxs * ncell);
    SplitBuffers()
    {
        for (size_t i = 0; i < disp.size() / 3; ++i)
            for (int c = 0; c < 3; ++c) disp[3 * i + c] = 0.01f * (float)((i * 7 + c) % 3);
    }
};

static void host_calls(SplitBuffers& z, bool expect_ok)
{
    const double frac[12] = {0, 0, 0, 0, .5, .5, .5, 0, .5, .5, .5, 0};
    const double b[4] = {1, .7, .7, .7};
    dsx_plan_info info;
    dsx_model_desc d = fcc_desc(frac, b, 5);
    dsx_status s = dsx_plan_query(&d, &info);
    CHECK(s == DSX_OK || (!expect_ok && s == DSX_ERR_NOMEM));
    if (s == DSX_OK) CHECK(info.fields_per_site == 55);
    d.n[1] = 0;
    s = dsx_plan_query(&d, &info);
    CHECK(s == DSX_ERR_ARG || (!expect_ok && s == DSX_ERR_NOMEM));
    CHECK(dsx_last_error() != nullptr);
    // split sites: 2 configurations, 4 sites, 3 distinct displacements per site
    const int n[3] = {3, 4, 2};
    int32_t ns = 0;
    s = dsx_split_sites(n, z.S, frac, b, z.M, z.occ.data(), z.disp.data(), 0.0, z.maxs, &ns, z.fo.data(),
                        z.bo.data(), z.po.data(), z.oo.data());
    CHECK(s == DSX_OK || (!expect_ok && s == DSX_ERR_NOMEM));
    if (s == DSX_OK) CHECK(ns >= z.S && ns <= 3 * z.S);
    s = dsx_split_sites(n, z.S, frac, b, z.M, z.occ.data(), z.disp.data(), 0.0, 2, &ns, z.fo.data(), z.bo.data(),
                        z.po.data(), z.oo.data());
    CHECK(s == DSX_ERR_UNSUPPORTED || (!expect_ok && s == DSX_ERR_NOMEM));
    s = dsx_split_sites(n, z.S, frac, b, z.M, z.occ.data(), nullptr, 0.0, z.maxs, &ns, z.fo.data(), z.bo.data(),
                        z.po.data(), z.oo.data());
    CHECK(s == DSX_ERR_ARG);
}

int main()
{
    arena_stress();
    SplitBuffers z;
    host_calls(z, true);
    // every allocation of the host calls failing in turn
    int k = 0;
    for (; k < 10000; ++k) {
        g_fail_after = k;
        host_calls(z, false);
        const bool finished = g_fail_after > 0;   // allocations left over: the calls completed
        g_fail_after = -1;
        if (finished) break;
    }
    CHECK(k < 10000);
    host_calls(z, true);
    std::printf("host runtime checks passed (%d allocation failure points)\n", k);
    return 0;
}
