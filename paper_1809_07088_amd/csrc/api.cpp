// Host runtime of the dsx C-ABI: model manager, planner and launch sequencing.
//
// A model owns its device state:
//   inputs   occ [M][S][ncell], vec [M][S][ncell][3] (displacements or spins)
//   sums     float64 lattice sums [M][S][T] (the k = 0 coefficients)
//   spectra  complex64 k-major half spectra X [M][k1][k2][S*F][n3/2+1]
//   tables   float64-generated phase tables for each output box in use
// compute_intensity / noise_filter enqueue, on the caller's stream:
//   sums -> plane FFTs (generation + axes 3, 2) -> axis-1 FFT    (when the sites changed)
//   recombination over the box -> float64 Bragg points -> [Lanczos filter]
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <array>
#include <climits>
#include <map>
#include <tuple>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "dsx.h"
#include "dsx_internal.h"
#include "arena.h"

using namespace dsx;

namespace {

thread_local std::string g_err;

void dfree(void* p) { if (p) (void)hipFree(p); }

dsx_status fail(dsx_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

// Host failures (allocation, thread creation) never cross the C-ABI as exceptions: every
// entry point runs its body through guarded(), which turns them into DSX_ERR_NOMEM.
template <typename F>
dsx_status guarded(F&& f) noexcept
{
    try {
        return f();
    } catch (...) {
        try {
            g_err = "host allocation or resource failure";
        } catch (...) {
            g_err.clear();
        }
        return DSX_ERR_NOMEM;
    }
}

// ---------------------------------------------------------------------------- instrumentation
struct Prof {
    std::mutex mu;
    bool on = false;
    std::string only;   // when not empty, the one kernel kind that is timed
    struct Pending { std::string name; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<long long, double>> stats;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
Prof g_prof;

// Records an event before and after the launch `fn` on stream st when enabled.
template <typename Fn>
hipError_t timed(const char* name, hipStream_t st, Fn fn)
{
    if (g_recorder) {            // a batch records its launches: label them with the step
        g_recorder->stage = name;
        return fn();
    }
    if (!g_prof.on) return fn();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.only.empty() && g_prof.only != name) return fn();
        a = g_prof.get();
        b = g_prof.get();
    }
    if (!a || !b) return fn();
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({name, a, b});
    return hipSuccess;
}

struct Box {
    int g0[3];
    int cnt[3];
    int half = 0;   // symmetric box stored as its planes G1 <= 0 only (I(-G) = I(G))
    bool operator<(const Box& o) const {
        for (int a = 0; a < 3; ++a) {
            if (g0[a] != o.g0[a]) return g0[a] < o.g0[a];
            if (cnt[a] != o.cnt[a]) return cnt[a] < o.cnt[a];
        }
        return half < o.half;
    }
};

bool symmetric_box(const Box& b)
{
    for (int a = 0; a < 3; ++a)
        if (b.cnt[a] % 2 == 0 || b.g0[a] != -(b.cnt[a] - 1) / 2) return false;
    return true;
}

int stored_planes(const Box& b) { return b.half ? (b.cnt[0] + 1) / 2 : b.cnt[0]; }

long floordiv_l(long a, long b) { long q = a / b; if ((a % b) != 0 && a < 0) --q; return q; }
long ceildiv_l(long a, long b) { return -floordiv_l(-a, b); }

// H count of residue k on an axis (g0 <= k + n H < g0 + cnt)
int hcount(int k, int n, int g0, int cnt)
{
    const long lo = ceildiv_l((long)g0 - k, n);
    const long hi = floordiv_l((long)g0 + cnt - 1 - k, n);
    return hi >= lo ? (int)(hi - lo + 1) : 0;
}

AxisPlan make_plan(int n)
{
    AxisPlan p{};
    p.n = n;
    int r = n;
    // primes above 5 first: the first pass of a Stockham transform needs no twiddles
    for (int f = 7; f <= r; f += 2) {
        if (f % 3 == 0 || f % 5 == 0) continue;
        while (r % f == 0) { p.rad[p.nrad++] = f; r /= f; }
    }
    while (r % 4 == 0) { p.rad[p.nrad++] = 4; r /= 4; }
    while (r % 2 == 0) { p.rad[p.nrad++] = 2; r /= 2; }
    for (int f : {3, 5}) while (r % f == 0) { p.rad[p.nrad++] = f; r /= f; }
    return p;
}

// Is `p` a valid radix sequence for its length: radices 2, 4 or odd (>= 3), product n.
bool plan_valid(const AxisPlan& p)
{
    if (p.n < 1 || p.nrad < 0 || p.nrad > kMaxRadices) return false;
    long prod = 1;
    for (int i = 0; i < p.nrad; ++i) {
        const int r = p.rad[i];
        if (!(r == 2 || r == 4 || (r >= 3 && (r & 1)))) return false;
        prod *= r;
        if (prod > p.n) return false;
    }
    return prod == p.n;
}

// Radix sequences of length n for the autotuner: the default first, then every order of
// every grouping of the factor 2^a into 4s and 2s with the odd primes, at most `cap`.
std::vector<AxisPlan> plan_candidates(int n, int cap)
{
    std::vector<AxisPlan> out{make_plan(n)};
    std::vector<int> odd;
    int r = n, twos = 0;
    while (r % 2 == 0) { ++twos; r /= 2; }
    for (int f = 3; f <= r; f += 2)
        while (r % f == 0) { odd.push_back(f); r /= f; }
    for (int fours = twos / 2; fours >= 0 && (int)out.size() < cap; --fours) {
        std::vector<int> rs(odd);
        rs.insert(rs.end(), fours, 4);
        rs.insert(rs.end(), twos - 2 * fours, 2);
        if ((int)rs.size() > kMaxRadices) continue;
        std::sort(rs.begin(), rs.end());
        do {
            AxisPlan p{};
            p.n = n;
            p.nrad = (int)rs.size();
            for (size_t i = 0; i < rs.size(); ++i) p.rad[i] = rs[i];
            bool dup = false;
            for (const AxisPlan& q : out)
                dup = dup || (q.nrad == p.nrad && std::equal(q.rad, q.rad + q.nrad, p.rad));
            if (!dup) out.push_back(p);
        } while ((int)out.size() < cap && std::next_permutation(rs.begin(), rs.end()));
    }
    return out;
}

std::string plan_string(const AxisPlan& p)
{
    std::string s;
    for (int i = 0; i < p.nrad; ++i) s += (i ? "x" : "") + std::to_string(p.rad[i]);
    return s.empty() ? "1" : s;
}

bool parse_plan(const std::string& s, int n, AxisPlan* out)
{
    AxisPlan p{};
    p.n = n;
    std::istringstream in(s);
    std::string tok;
    while (std::getline(in, tok, 'x')) {
        if (tok.empty() || p.nrad >= kMaxRadices) return false;
        const int v = std::atoi(tok.c_str());
        if (v == 1 && s == "1") break;
        p.rad[p.nrad++] = v;
    }
    if (!plan_valid(p)) return false;
    *out = p;
    return true;
}

// Rows a*, b*, c* of the reciprocal basis (a* = 2 pi b x c / V), a along x and b in
// the xy plane.  Returns false for an invalid cell.
bool reciprocal_basis(const double cell[6], double out[9])
{
    const double d2r = M_PI / 180.0;
    const double a = cell[0], b = cell[1], c = cell[2];
    const double al = cell[3] * d2r, be = cell[4] * d2r, ga = cell[5] * d2r;
    if (!(a > 0 && b > 0 && c > 0) || !(al > 0 && be > 0 && ga > 0 && al < M_PI && be < M_PI && ga < M_PI))
        return false;
    const double A[3] = {a, 0.0, 0.0};
    const double B[3] = {b * std::cos(ga), b * std::sin(ga), 0.0};
    const double cx = c * std::cos(be);
    const double cy = c * (std::cos(al) - std::cos(be) * std::cos(ga)) / std::sin(ga);
    const double cz2 = c * c - cx * cx - cy * cy;
    if (!(cz2 > 0)) return false;
    const double C[3] = {cx, cy, std::sqrt(cz2)};
    auto cross = [](const double* u, const double* v, double* w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double bc[3], ca[3], ab[3];
    cross(B, C, bc); cross(C, A, ca); cross(A, B, ab);
    const double V = A[0] * bc[0] + A[1] * bc[1] + A[2] * bc[2];
    if (!(V > 0)) return false;
    for (int i = 0; i < 3; ++i) {
        out[i] = 2 * M_PI * bc[i] / V;
        out[3 + i] = 2 * M_PI * ca[i] / V;
        out[6 + i] = 2 * M_PI * ab[i] / V;
    }
    return true;
}

float2 cis(double x)   // e^{2 pi i x}, argument reduced mod 1 in float64 first
{
    x -= std::floor(x);
    return make_float2((float)std::cos(2 * M_PI * x), (float)std::sin(2 * M_PI * x));
}

struct DeviceTables {
    float2* tab1 = nullptr;
    float2* tab2 = nullptr;
    float2* tabK2 = nullptr;
    float2* tabK3 = nullptr;
    float2* tabH3 = nullptr;
    int4* work = nullptr;
    int4* work2 = nullptr;     // the same blocks with two G1 planes of one column each
    int4* work3 = nullptr;     // work2 with each block cut into k3 slices (null: no slicing)
    int2* k3tab = nullptr;     // [n3] (H3lo, count) of residue k3 in the box
    int hmin_all = 0;          // fewest H3 values of any (k3, chunk) item ...
    int hmin_slice[8] = {};    // ... and of any item of one k3 slice
    int H3min = 0, nH3span = 0;
    int nwork = 0, nwork2 = 0, nwork3 = 0, hc = 0, nchunk3 = 0, block = 0;
    int n3s = 0, block3 = 0;   // k3 per slice, threads per plane of a sliced block
    int4* work_mr = nullptr;   // magnetic models: blocks of the row-staged form (null: not used)
    int nwork_mr = 0, rows_mr = 0, csites_mr = 0, qmod_mr = 0, qmod2_mr = 0, qmod1_mr = 0;
};

// Releases every device buffer of one cached box.
void free_tables(DeviceTables& t)
{
    dfree(t.tab1); dfree(t.tab2); dfree(t.tabK2); dfree(t.tabK3); dfree(t.tabH3);
    dfree(t.work); dfree(t.work2); dfree(t.work3); dfree(t.k3tab); dfree(t.work_mr);
    t = DeviceTables{};
}

struct LaunchPlan {
    RecombParams rp;
    bool mag_rows = false;     // the row-staged magnetic form
    bool direct = false;       // the direct form (order 0)
    int hc = 0, block = 0;
    size_t lds = 0;
    BraggParams bp;
};

}  // namespace

struct dsx_model_s {
    // description
    double cell[6];
    int n[3];
    int S, kind, has_occ, order, M;
    double normN;
    std::vector<double> frac, b, ff;
    bool has_ff = false;
    double recip[9];
    // plan
    int F = 0, T = 0, first_mono = 0, nh = 0, SF = 0, ncell = 0, nclass = 0;
    std::vector<int> site_of, class_of;     // class-sorted site order
    std::vector<int> sc_start;              // site chunks for the recombination LDS budget
    size_t chunk_lds = 0;
    int bs_elems = 0, xs_elems = 0;
    AxisPlan plan[3];
    // device state
    int device = 0;
    float* d_occ = nullptr;
    float* d_vec = nullptr;
    // magnetic models with displacements: the Debye-Waller factor of Eq. dw
    int dw_order = 0;              // Taylor order of T_mu(G); 0 = no displacements (T = 1)
    int dwT = 0;                   // monomials of that order
    float* d_dsp = nullptr;        // [M][S][ncell][3] fractional displacements
    double* d_dwsums = nullptr;    // [M*S][dwT] float64 lattice sums of the displacement monomials
    double* d_dwc = nullptr;       // [S][dwT] their means over occupied atoms and configurations
    double* d_partial = nullptr;
    double* d_sums = nullptr;
    double* d_site = nullptr;   // [S][11]: r_mu, b_mu, form factor
    float2* d_X = nullptr;
    float2* d_tw[3] = {nullptr, nullptr, nullptr};
    float* d_ext = nullptr;   size_t ext_cap = 0;
    float* d_pts = nullptr;   size_t pts_cap = 0;   // I(G) on the box of a point list's windows
    double* d_q = nullptr;    size_t q_cap = 0;     // the point list
    float* d_stage = nullptr; size_t stage_cap = 0;
    std::map<Box, DeviceTables> tables;
    std::map<std::tuple<int, int, int>, float*> lanczos_w;   // (m, m', s) -> weights
    int sum_chunk = 256, sum_chunks = 0;   // cells per sums block, blocks per (config, site)
    // plan knobs (defaults, or chosen by the autotuner for this model's key)
    int tune_recomb_variant = 0;   // 0 default form, 2 class form, 3 unfolded, 4 unsliced, 5 direct
    int tune_fchunk = 0;           // fields per FFT plane block (0 = heuristic)
    int tune_lanczos_t1 = 12;      // planes per filter block
    int tune_tc = 0;               // columns per block of the LDS axis-1 FFT (0 = heuristic)
    bool tuned = false;
    // state
    std::vector<char> set;
    bool dirty = true;
    bool failed = false;
    bool grid_set = false;
    Box box{};
    hipStream_t last_stream = nullptr;   // stream of the last enqueued work
    hipEvent_t order_ev = nullptr;       // orders work across the caller's streams
    int pins = 0;                        // batches that recorded this model's buffers
    // served models: spectra, partial sums and the grown box live in the server's
    // arena for the duration of one request; everything else stays resident
    dsx_server_s* server = nullptr;
    std::atomic<int> queued{0};          // requests submitted and not yet finished
    size_t spectrum_bytes = 0, partial_bytes = 0;
};

namespace {

#define HIPCHK(m, expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            if (m) (m)->failed = true;                                                         \
            return fail(DSX_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
        }                                                                                      \
    } while (0)

dsx_status validate_desc(const dsx_model_desc* d)
{
    if (!d) return fail(DSX_ERR_ARG, "desc is NULL");
    for (int a = 0; a < 3; ++a)
        if (d->n[a] < 1) return fail(DSX_ERR_ARG, "n must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (d->n[a] > DSX_MAX_N) return fail(DSX_ERR_UNSUPPORTED, "n exceeds DSX_MAX_N");
    if (d->n_sites < 1) return fail(DSX_ERR_ARG, "n_sites must be >= 1");
    if (d->n_sites > DSX_MAX_SITES) return fail(DSX_ERR_UNSUPPORTED, "n_sites exceeds DSX_MAX_SITES");
    if (!d->frac || !d->b) return fail(DSX_ERR_ARG, "frac and b are required");
    if (d->kind != DSX_NUCLEAR && d->kind != DSX_MAGNETIC) return fail(DSX_ERR_ARG, "bad kind");
    if (d->taylor_order < 0) return fail(DSX_ERR_ARG, "taylor_order must be >= 0");
    if (d->taylor_order > DSX_MAX_ORDER) return fail(DSX_ERR_UNSUPPORTED, "taylor_order exceeds DSX_MAX_ORDER");
    if (d->n_configs < 1) return fail(DSX_ERR_ARG, "n_configs must be >= 1");
    if (!(d->norm_N >= 0.0)) return fail(DSX_ERR_ARG, "norm_N must be >= 0");
    if (d->kind == DSX_NUCLEAR && d->taylor_order == 0 && !d->has_occ)
        return fail(DSX_ERR_ARG, "a nuclear model needs occupancies or displacements");
    double rb[9];
    if (!reciprocal_basis(d->cell, rb)) return fail(DSX_ERR_ARG, "invalid cell");
    for (int i = 0; i < 3 * d->n_sites; ++i)
        if (!std::isfinite(d->frac[i])) return fail(DSX_ERR_ARG, "non-finite site position");
    return DSX_OK;
}

// Sizes shared by plan_query and create_model.
struct Sizes {
    int F, T, first_mono, nh, ncell, nclass;
    long long spectrum_bytes, device_bytes;
};

int count_classes(const dsx_model_desc* d, std::vector<int>* site_of, std::vector<int>* class_of)
{
    // group sites sharing r_mu3 (and, for magnetic models, the form factor)
    std::vector<int> cls(d->n_sites, -1);
    int nc = 0;
    for (int i = 0; i < d->n_sites; ++i) {
        if (cls[i] >= 0) continue;
        cls[i] = nc;
        for (int j = i + 1; j < d->n_sites; ++j) {
            if (cls[j] >= 0) continue;
            bool same = d->frac[3 * i + 2] == d->frac[3 * j + 2];
            if (same && d->ff)
                for (int k = 0; k < 7; ++k) same = same && d->ff[7 * i + k] == d->ff[7 * j + k];
            if (same) cls[j] = nc;
        }
        ++nc;
    }
    if (site_of && class_of) {
        site_of->clear(); class_of->clear();
        for (int c = 0; c < nc; ++c)
            for (int i = 0; i < d->n_sites; ++i)
                if (cls[i] == c) { site_of->push_back(i); class_of->push_back(c); }
    }
    return nc;
}

Sizes sizes_of(const dsx_model_desc* d)
{
    Sizes z{};
    z.ncell = d->n[0] * d->n[1] * d->n[2];
    z.nh = d->n[2] / 2 + 1;
    if (d->kind == DSX_MAGNETIC) { z.T = 3; z.F = 3; z.first_mono = 0; }
    else {
        z.T = n_monomials(d->taylor_order);
        z.first_mono = d->has_occ ? 0 : 1;
        z.F = z.T - z.first_mono;
    }
    z.nclass = count_classes(d, nullptr, nullptr);
    const long long M = d->n_configs, S = d->n_sites;
    z.spectrum_bytes = M * d->n[0] * d->n[1] * S * z.F * (long long)z.nh * 8;
    long long in = 0;
    if (d->has_occ) in += M * S * z.ncell * 4;
    if (d->kind == DSX_MAGNETIC || d->taylor_order > 0) in += M * S * z.ncell * 12;
    const long long sc = sums_chunk(z.ncell, M * S);
    const long long chunks = (z.ncell + sc - 1) / sc;
    z.device_bytes = z.spectrum_bytes + in + M * S * z.T * 8 * (chunks + 1);
    if (d->kind == DSX_MAGNETIC && d->taylor_order > 0) {
        // displacements, their lattice sums (partials shared with the spins') and means
        const long long dwT = n_monomials(d->taylor_order);
        z.device_bytes += M * S * z.ncell * 12 + M * S * dwT * 8 * (chunks > 1 ? chunks : 1)
                        + M * S * dwT * 8 + S * dwT * 8;
    }
    return z;
}

dsx_status check_model(dsx_model m)
{
    if (!m) return fail(DSX_ERR_ARG, "model is NULL");
    if (m->failed) return fail(DSX_ERR_DEVICE, "model is in a failed state after a device error");
    return DSX_OK;
}

void free_model(dsx_model m)
{
    dfree(m->d_occ); dfree(m->d_vec); dfree(m->d_partial); dfree(m->d_sums); dfree(m->d_X);
    dfree(m->d_dsp); dfree(m->d_dwsums); dfree(m->d_dwc);
    dfree(m->d_site);
    for (auto& t : m->d_tw) dfree(t);
    dfree(m->d_ext); dfree(m->d_stage); dfree(m->d_pts); dfree(m->d_q);
    for (auto& kv : m->tables) free_tables(kv.second);
    for (auto& kv : m->lanczos_w) dfree(kv.second);
    if (m->order_ev) (void)hipEventDestroy(m->order_ev);
}

// Calls on one model are serialised: work enqueued on st starts after everything the
// model enqueued before, on whichever stream that was.
dsx_status follow(dsx_model m, hipStream_t st)
{
    if (m->last_stream != st) {
        HIPCHK(m, hipEventRecord(m->order_ev, m->last_stream));
        HIPCHK(m, hipStreamWaitEvent(st, m->order_ev, 0));
    }
    m->last_stream = st;
    return DSX_OK;
}

dsx_status tables_for(dsx_model m, const Box& bx, DeviceTables** out)
{
    auto it = m->tables.find(bx);
    if (it != m->tables.end()) { *out = &it->second; return DSX_OK; }
    if (m->tables.size() >= 8 && m->pins == 0) {   // keep the cache small: drop every cached box
        // but the grid's own (never while a recorded batch still points at a cached table)
        hipError_t se = hipStreamSynchronize(m->last_stream);
        if (se != hipSuccess) { m->failed = true; return fail(DSX_ERR_DEVICE, hipGetErrorString(se)); }
        for (auto it = m->tables.begin(); it != m->tables.end();) {
            if (m->grid_set && !(it->first < m->box) && !(m->box < it->first)) { ++it; continue; }
            free_tables(it->second);
            it = m->tables.erase(it);
        }
    }
    DeviceTables t;
    const int S = m->S, n1 = m->n[0], n2 = m->n[1], n3 = m->n[2];
    std::vector<float2> t1((size_t)S * bx.cnt[0]), t2((size_t)S * bx.cnt[1]), tk((size_t)S * n3);
    std::vector<float2> tk2((size_t)S * n2);
    for (int mu = 0; mu < S; ++mu) {
        for (int k = 0; k < n2; ++k)
            tk2[(size_t)mu * n2 + k] = cis((double)k / n2 * m->frac[3 * mu + 1]);
        for (int i = 0; i < bx.cnt[1]; ++i)
            t2[(size_t)mu * bx.cnt[1] + i] = cis((double)(bx.g0[1] + i) / n2 * m->frac[3 * mu + 1]);
        for (int k = 0; k < n3; ++k)
            tk[(size_t)mu * n3 + k] = cis((double)k / n3 * m->frac[3 * mu + 2]);
    }
    // b folded in tab1 must be computed in float64 before rounding
    for (int mu = 0; mu < S; ++mu)
        for (int i = 0; i < bx.cnt[0]; ++i) {
            double x = (double)(bx.g0[0] + i) / n1 * m->frac[3 * mu];
            x -= std::floor(x);
            t1[(size_t)mu * bx.cnt[0] + i] = make_float2((float)(m->b[mu] * std::cos(2 * M_PI * x)),
                                                         (float)(m->b[mu] * std::sin(2 * M_PI * x)));
        }
    t.H3min = (int)floordiv_l(bx.g0[2], n3);
    const int H3max = (int)floordiv_l((long)bx.g0[2] + bx.cnt[2] - 1, n3);
    t.nH3span = H3max - t.H3min + 1;
    std::vector<float2> th((size_t)m->nclass * t.nH3span);
    for (int c = 0; c < m->nclass; ++c) {
        int mu = -1;
        for (size_t i = 0; i < m->site_of.size(); ++i)
            if (m->class_of[i] == c) { mu = m->site_of[i]; break; }
        for (int h = 0; h < t.nH3span; ++h)
            th[(size_t)c * t.nH3span + h] = cis((double)(t.H3min + h) * m->frac[3 * mu + 2]);
    }
    // ---- work list of the recombination: (k1, k2, G1, H2 range), one block each
    const bool mag = m->kind == DSX_MAGNETIC;
    int maxH2 = 0, maxH3 = 0;
    for (int k = 0; k < n2; ++k) maxH2 = std::max(maxH2, hcount(k, n2, bx.g0[1], bx.cnt[1]));
    for (int k = 0; k < n3; ++k) maxH3 = std::max(maxH3, hcount(k, n3, bx.g0[2], bx.cnt[2]));
    const int hcs_nuc[4] = {4, 8, 17, 32};
    const int hcs_mag[3] = {4, 8, 17};
    const int* hcs = mag ? hcs_mag : hcs_nuc;
    // orders above kMaxOrderFast have runs of at most 8 H3 per thread
    const int nhcs = mag ? 3 : (m->order > kMaxOrderFast ? 2 : 4);
    t.hc = hcs[nhcs - 1];
    for (int i = 0; i < nhcs; ++i) if (hcs[i] >= maxH3) { t.hc = hcs[i]; break; }
    t.nchunk3 = (maxH3 + t.hc - 1) / t.hc;
    const int maxT = recombine_max_threads(t.hc, mag);
    const int per_h2 = n3 * t.nchunk3;
    if (per_h2 > maxT) return fail(DSX_ERR_UNSUPPORTED, "output box too long along axis 3 for this supercell");
    if (maxH2 > 4095) return fail(DSX_ERR_UNSUPPORTED, "output box too long along axis 2 for this supercell");
    if ((size_t)m->nclass * t.nH3span * sizeof(float2) > 32 * 1024)
        return fail(DSX_ERR_UNSUPPORTED, "output box too long along axis 3 for this supercell");
    const int h2per = std::max(1, maxT / per_h2);
    const bool friedel = symmetric_box(bx);
    if (bx.half && !friedel) return fail(DSX_ERR_STATE, "half storage needs a symmetric box");
    std::vector<std::pair<long long, int4>> items, items2, items3, items_mr;
    int maxrows = 1;
    // the row-staged magnetic form: one thread per G3 of the box (at most
    // kMagRowsMaxThreads), rows per block from the LDS budget (about four blocks per CU),
    // site chunks of the staging area, and the H3 residues the classes are summed over
    if (mag && bx.cnt[2] <= kMagRowsMaxThreads) {
        const int NC = m->nclass;
        int q = 0;
        bool uniform = true;
        for (int i = 0; i < S && m->has_ff; ++i)
            for (int k = 0; k < 7; ++k) uniform = uniform && m->ff[8 * m->site_of[i] + k] == m->ff[8 * m->site_of[0] + k];
        if (uniform && NC <= kMagRowsMaxClasses)
            for (int cand : {1, 2, 3, 4, 6, 8}) {
                bool ok = true;
                for (int i = 0; i < S && ok; ++i) {
                    const double x = m->frac[3 * m->site_of[i] + 2] * cand;
                    ok = std::fabs(x - std::round(x)) < 1e-9;
                }
                if (ok) { q = cand <= NC ? cand : 0; break; }
            }
        t.qmod_mr = q;
        // rows whose H2 agree modulo q2 (every r_mu2 a multiple of 1/q2) share their site
        // phases e^{2 pi i g2 r_mu2}, so a block stages min(rows, q2) of them only; planes
        // whose H1 agree modulo q1 share e^{2 pi i g1 r_mu1}, and one block serves up to four
        // of them (one configuration: the sums of several are accumulated per row)
        auto grid_of = [&](int axis) {
            for (int cand : {1, 2, 3, 4, 6, 8}) {
                bool ok = true;
                for (int i = 0; i < S && ok; ++i) {
                    const double x = m->frac[3 * m->site_of[i] + axis] * cand;
                    ok = std::fabs(x - std::round(x)) < 1e-9;
                }
                if (ok) return cand;
            }
            return 0;
        };
        const int q2 = grid_of(1);
        t.qmod2_mr = q2;
        t.qmod1_mr = m->M == 1 ? grid_of(0) : 0;
        int cs = S;
        while (cs > 1 && (size_t)cs * 3 * n3 * sizeof(float2) > 12 * 1024) cs = (cs + 1) / 2;
        const size_t budget = 48 * 1024 / sizeof(float2);
        const size_t fixed = magnetic_rows_lds_elems(0, cs, S, NC, n3, t.nH3span);
        const size_t per_row = magnetic_rows_lds_elems(1, 0, S, NC, n3, 0) - (size_t)S * n3;
        // residue rows: every row of a column in one block when q2 staged rows fit; else the
        // rows are staged one by one, as many as fit
        if (q2 > 0 && fixed + std::min(q2, kMagRowsMaxRows) * per_row > budget) t.qmod2_mr = 0;
        int rows;
        if (t.qmod2_mr > 0)
            rows = kMagRowsMaxRows;
        else
            rows = fixed < budget ? (int)((budget - fixed) / per_row) : 0;
        rows = std::min(std::min(rows, kMagRowsMaxRows), maxH2);
        if (rows >= 1) { t.rows_mr = rows; t.csites_mr = cs; }
    }
    // k3 slices of the two-plane blocks: halves of the k3 range when it is long enough
    // that a slice still writes 64-byte runs of an output row
    const int nsl = (n3 >= 16) ? 2 : 1;
    t.n3s = (n3 + nsl - 1) / nsl;
    for (int k1 = 0; k1 < n1; ++k1) {
        const int nH1 = hcount(k1, n1, bx.g0[0], bx.cnt[0]);
        const int H1lo = (int)ceildiv_l((long)bx.g0[0] - k1, n1);
        for (int k2 = 0; k2 < n2; ++k2) {
            const int nH2 = hcount(k2, n2, bx.g0[1], bx.cnt[1]);
            if (nH2 == 0) continue;
            const int km1 = (n1 - k1) % n1, km2 = (n2 - k2) % n2;
            // order key: a column and its mirror are adjacent
            const long long c0 = (long long)k1 * n2 + k2, c1 = (long long)km1 * n2 + km2;
            const long long key = std::min(c0, c1) * 2 + (c0 > c1 ? 1 : 0);
            const int np = (nH2 + h2per - 1) / h2per;
            const int rpp = (nH2 + np - 1) / np;
            std::vector<std::pair<int, int>> planes;   // (j1, mirror) of the G1 planes computed
            for (int j1 = 0; j1 < nH1; ++j1) {
                const int G1 = k1 + n1 * (H1lo + j1);
                int mirror = 0;
                if (friedel) {
                    if (G1 > 0) continue;
                    if (G1 == 0) {
                        if (k2 > km2) continue;
                        mirror = k2 < km2 ? 1 : 0;
                    } else {
                        mirror = bx.half ? 0 : 1;   // half storage keeps the planes G1 <= 0 only
                    }
                }
                planes.push_back({j1, mirror});
            }
            if (t.rows_mr > 0) {
                const int npm = (nH2 + t.rows_mr - 1) / t.rows_mr;
                const int rpm = (nH2 + npm - 1) / npm;
                // planes grouped by the residue of H1 mod q1, at most four a group, in H1 order
                std::vector<std::vector<std::pair<int, int>>> groups;
                if (t.qmod1_mr > 0) {
                    const int q1 = t.qmod1_mr;
                    for (int res = 0; res < q1; ++res) {
                        std::vector<std::pair<int, int>> g;
                        for (const auto& pl : planes)
                            if (pl.first % q1 == res) {
                                // a group's planes are j1, j1 + q1, ... (the kernel steps G1 by q1 n1)
                                if (g.size() == 4 || (!g.empty() && pl.first != g.back().first + q1)) {
                                    groups.push_back(g);
                                    g.clear();
                                }
                                g.push_back(pl);
                            }
                        if (!g.empty()) groups.push_back(g);
                    }
                } else {
                    for (const auto& pl : planes) groups.push_back({pl});
                }
                for (int part = 0; part < npm; ++part) {
                    const int h2a = part * rpm, h2b = std::min(nH2, h2a + rpm);
                    if (h2a >= h2b) continue;
                    for (const auto& g : groups) {
                        const int G1 = k1 + n1 * (H1lo + g[0].first);
                        int wv = h2a | (h2b << 12) | ((int)(g.size() - 1) << 28);
                        for (size_t p = 0; p < g.size(); ++p) wv |= g[p].second << (24 + p);
                        items_mr.push_back({key * 4096 + g[0].first, make_int4(k1, k2, G1, wv)});
                    }
                }
            }
            for (int part = 0; part < np; ++part) {
                const int h2a = part * rpp, h2b = std::min(nH2, h2a + rpp);
                if (h2a >= h2b) continue;
                maxrows = std::max(maxrows, h2b - h2a);
                for (size_t i = 0; i < planes.size(); ++i) {
                    const int j1 = planes[i].first;
                    const int G1 = k1 + n1 * (H1lo + j1);
                    items.push_back({key * 4096 + j1, make_int4(k1, k2, G1, h2a | (h2b << 12) | (planes[i].second << 24))});
                }
                // planes are consecutive in H1 (the skipped ones are all at the end)
                for (size_t i = 0; i < planes.size(); i += 2) {
                    const int j1 = planes[i].first;
                    const int G1 = k1 + n1 * (H1lo + j1);
                    const int hasb = i + 1 < planes.size() ? 1 : 0;
                    const int mb = hasb ? planes[i + 1].second : 0;
                    const int wv = h2a | (h2b << 12) | (planes[i].second << 24) | (hasb << 25) | (mb << 26);
                    items2.push_back({key * 4096 + j1, make_int4(k1, k2, G1, wv)});
                    // the slices of one block are adjacent: they share the column's spectra
                    // and the cache lines of the output rows
                    for (int sl = 0; sl < nsl && nsl > 1; ++sl)
                        items3.push_back({key * 4096 + j1, make_int4(k1, k2, G1, wv | (sl << 27))});
                }
            }
        }
    }
    // blocks are dealt round-robin to the 8 XCDs: XCD x runs the x-th contiguous eighth
    // of the list, in which the blocks of a column and of its mirror are adjacent
    auto xcd_order = [](std::vector<std::pair<long long, int4>>& its) {
        std::stable_sort(its.begin(), its.end(),
                         [](const std::pair<long long, int4>& x, const std::pair<long long, int4>& y) { return x.first < y.first; });
        const size_t per = (its.size() + 7) / 8;
        std::vector<int4> wl(8 * per, make_int4(-1, 0, 0, 0));
        for (size_t b = 0; b < wl.size(); ++b) {
            const size_t L = (b % 8) * per + b / 8;
            if (L < its.size()) wl[b] = its[L].second;
        }
        return wl;
    };
    const std::vector<int4> work = xcd_order(items), work2 = xcd_order(items2), work3 = xcd_order(items3);
    const std::vector<int4> work_mr = xcd_order(items_mr);
    t.nwork_mr = (int)work_mr.size();
    t.nwork = (int)work.size();
    t.nwork2 = (int)work2.size();
    t.nwork3 = (int)work3.size();
    t.block = ((std::min(maxT, maxrows * per_h2) + 63) / 64) * 64;
    t.block3 = ((std::min(maxT, maxrows * t.n3s * t.nchunk3) + 63) / 64) * 64;
    std::vector<int2> k3t(n3);
    t.hmin_all = t.hc;
    for (int s = 0; s < 8; ++s) t.hmin_slice[s] = t.hc;
    for (int k = 0; k < n3; ++k) {
        k3t[k] = make_int2((int)ceildiv_l((long)bx.g0[2] - k, n3), hcount(k, n3, bx.g0[2], bx.cnt[2]));
        for (int c = 0; c < t.nchunk3; ++c) {
            const int h = std::max(0, std::min(t.hc, k3t[k].y - c * t.hc));
            t.hmin_all = std::min(t.hmin_all, h);
            t.hmin_slice[k / t.n3s] = std::min(t.hmin_slice[k / t.n3s], h);
        }
    }

    auto up = [&](float2** dst, const std::vector<float2>& src) -> hipError_t {
        hipError_t e = hipMalloc(dst, sizeof(float2) * std::max<size_t>(1, src.size()));
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, src.data(), sizeof(float2) * src.size(), hipMemcpyHostToDevice);
    };
    hipError_t e;
    if ((e = up(&t.tab1, t1)) != hipSuccess || (e = up(&t.tab2, t2)) != hipSuccess ||
        (e = up(&t.tabK2, tk2)) != hipSuccess ||
        (e = up(&t.tabK3, tk)) != hipSuccess || (e = up(&t.tabH3, th)) != hipSuccess ||
        (e = hipMalloc(&t.work, sizeof(int4) * std::max<size_t>(1, work.size()))) != hipSuccess ||
        (e = hipMemcpy(t.work, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMalloc(&t.work2, sizeof(int4) * std::max<size_t>(1, work2.size()))) != hipSuccess ||
        (e = hipMemcpy(t.work2, work2.data(), sizeof(int4) * work2.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (!work3.empty() &&
         ((e = hipMalloc(&t.work3, sizeof(int4) * work3.size())) != hipSuccess ||
          (e = hipMemcpy(t.work3, work3.data(), sizeof(int4) * work3.size(), hipMemcpyHostToDevice)) != hipSuccess)) ||
        (!work_mr.empty() &&
         ((e = hipMalloc(&t.work_mr, sizeof(int4) * work_mr.size())) != hipSuccess ||
          (e = hipMemcpy(t.work_mr, work_mr.data(), sizeof(int4) * work_mr.size(), hipMemcpyHostToDevice)) != hipSuccess)) ||
        (e = hipMalloc(&t.k3tab, sizeof(int2) * k3t.size())) != hipSuccess ||
        (e = hipMemcpy(t.k3tab, k3t.data(), sizeof(int2) * k3t.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        free_tables(t);
        if (e == hipErrorOutOfMemory) return fail(DSX_ERR_NOMEM, "out of device memory for phase tables");
        m->failed = true;
        return fail(DSX_ERR_DEVICE, std::string("phase tables: ") + hipGetErrorString(e));
    }
    try {
        auto ins = m->tables.emplace(bx, t);
        *out = &ins.first->second;
    } catch (...) {
        free_tables(t);
        throw;
    }
    return DSX_OK;
}

// Memory layout of an output box: element (i1, i2, i3) at (i1 cnt1 + i2) pitch + i3 + off.
struct Layout {
    int pitch, off;
};

Layout dense_layout(const Box& b) { return Layout{b.cnt[2], 0}; }

// The direct form applies to nuclear models of Taylor order 0 with one field per site
// and no |Q|-dependent scattering factor.
bool direct_form_applies(dsx_model m)
{
    return m->kind == DSX_NUCLEAR && m->order == 0 && m->F == 1 && !m->has_ff;
}

dsx_status plan_recombine(dsx_model m, const Box& bx, float* out, const Layout& lay, LaunchPlan& lp)
{
    DeviceTables* tb = nullptr;
    dsx_status st = tables_for(m, bx, &tb);
    if (st != DSX_OK) return st;
    const int n1 = m->n[0], n2 = m->n[1], n3 = m->n[2];
    const bool mag = m->kind == DSX_MAGNETIC;
    if ((unsigned long long)bx.cnt[1] * lay.pitch * sizeof(float) >= (1ULL << 32))
        return fail(DSX_ERR_UNSUPPORTED, "one plane of the output box must stay below 4 GiB");
    RecombParams& p = lp.rp;
    std::memset(&p, 0, sizeof(p));
    p.X = m->d_X; p.out = out;
    p.tab1 = tb->tab1; p.tab2 = tb->tab2; p.tabK3 = tb->tabK3; p.tabH3 = tb->tabH3; p.tabK2 = tb->tabK2;
    p.n1 = n1; p.n2 = n2; p.n3 = n3; p.nh = m->nh; p.S = m->S; p.SF = m->SF; p.F = m->F; p.M = m->M;
    p.first_mono = m->first_mono;
    for (int a = 0; a < 3; ++a) {
        p.g0[a] = bx.g0[a]; p.cnt[a] = bx.cnt[a];
        p.tw[a] = 2.0 * M_PI / m->n[a];
    }
    p.opitch = lay.pitch; p.ooff = lay.off;
    p.ostream = (lay.pitch % 32 == 0 && lay.off % 32 == 0 && ((uintptr_t)out & 127) == 0) ? 1 : 0;
    p.H3min = tb->H3min; p.nH3span = tb->nH3span;
    p.nclass = m->nclass;
    p.work = tb->work; p.nwork = tb->nwork;
    p.nchunk3 = tb->nchunk3;
    {
        // DSX_RECOMBINE_VARIANT forces a kernel form (diagnostics and tests)
        const char* v = std::getenv("DSX_RECOMBINE_VARIANT");
        p.variant = (v && *v) ? std::atoi(v) : m->tune_recomb_variant;
    }
    p.nsc = (int)m->sc_start.size() - 1;
    for (size_t i = 0; i < m->sc_start.size(); ++i) p.sc_start[i] = m->sc_start[i];
    for (int i = 0; i < m->S; ++i) { p.site_of[i] = m->site_of[i]; p.class_of[i] = m->class_of[i]; }
    p.bs_elems = m->bs_elems;
    p.xs_elems = m->xs_elems;
    // parity form: every r_mu3 a multiple of 1/2 (exactly, as given); a |Q|-dependent
    // nuclear scattering factor needs the classes apart at level C (class form)
    p.nuc_ff = (m->kind == DSX_NUCLEAR && m->has_ff) ? 1 : 0;
    p.parity = (m->kind == DSX_NUCLEAR && !p.nuc_ff && m->order <= kMaxOrderFast) ? 1 : 0;
    for (int i = 0; i < m->S; ++i) {
        const double t2 = 2.0 * m->frac[3 * m->site_of[i] + 2];
        if (t2 != std::floor(t2)) p.parity = 0;
        const long a2 = (long)std::floor(t2);
        p.class_sign[m->class_of[i]] = (a2 % 2 == 0) ? 1 : -1;
    }
    const double C = mag ? 0.07265 : 1.0;
    p.scale = (float)(C / (m->normN * m->M));
    for (int i = 0; i < 9; ++i) p.recip[i] = (float)m->recip[i];
    p.ff_uniform = 1;
    for (int i = 0; i < m->S; ++i) {
        const int mu = m->site_of[i];
        for (int k = 0; k < 8; ++k) {
            p.ff[i][k] = m->has_ff ? (float)m->ff[8 * mu + k] : (k == 6 ? 1.f : 0.f);
            if (m->has_ff && m->ff[8 * mu + k] != m->ff[k]) p.ff_uniform = 0;
        }
    }
    {
        const double* R = m->recip;
        auto dot = [R](int a, int b) { return R[3 * a] * R[3 * b] + R[3 * a + 1] * R[3 * b + 1] + R[3 * a + 2] * R[3 * b + 2]; };
        const double tol = 1e-12 * dot(1, 1);
        p.ff_sep = (p.ff_uniform && std::fabs(dot(0, 1)) <= tol * std::sqrt(dot(0, 0) / dot(1, 1)) &&
                    std::fabs(dot(2, 1)) <= tol * std::sqrt(dot(2, 2) / dot(1, 1))) ? 1 : 0;
    }
    if (m->dw_order > 0) {
        p.dwc = m->d_dwc;
        p.dw_order = m->dw_order;
        p.dwT = m->dwT;
        p.dw_elems = m->S * n_pairs(m->dw_order);
    }
    lp.hc = tb->hc;
    lp.block = tb->block;
    lp.lds = m->chunk_lds + sizeof(float2) * ((size_t)m->nclass * tb->nH3span + p.dw_elems);
    {
        int c = 0;
        for (int i = 0; i < m->S; ++i)
            while (c <= m->class_of[i]) p.class_start[c++] = i;
        while (c <= m->nclass) p.class_start[c++] = m->S;
    }
    if (mag && m->dw_order == 0 && tb->work_mr) {
        lp.mag_rows = true;
        p.work = tb->work_mr;
        p.nwork = tb->nwork_mr;
        p.rows = tb->rows_mr;
        p.csites = tb->csites_mr;
        p.qmod = tb->qmod_mr;
        p.qmod2 = tb->qmod2_mr;
        p.qmod1 = tb->qmod1_mr;
        lp.block = std::max(64, (bx.cnt[2] + 63) / 64 * 64);
        const int staged = tb->qmod2_mr > 0 ? std::min(tb->rows_mr, tb->qmod2_mr) : tb->rows_mr;
        lp.lds = sizeof(float2) * magnetic_rows_lds_elems(staged, tb->csites_mr, m->S, m->nclass, n3, tb->nH3span);
    }
    // direct form: asked for, or by default where the levelled forms would spend their
    // blocks on set-up (one or two sites x configurations)
    if (direct_form_applies(m) && (p.variant == 5 || (p.variant == 0 && m->S * m->M <= 2)) &&
        (unsigned long long)bx.cnt[0] * bx.cnt[1] * bx.cnt[2] < (1ULL << 31)) {
        lp.direct = true;
        lp.lds = 0;
        p.planes = stored_planes(bx);   // a half-stored box: its planes G1 <= 0 only
    }
    if (lp.lds > 160 * 1024) return fail(DSX_ERR_UNSUPPORTED, "recombination does not fit the LDS for this box");
    // folded form: every r_mu2 a multiple of 1/2 (exactly, as given), fewer r3 classes
    // than sites, and the class buffers fit the LDS
    // (the folded kernel addresses the spectra of one configuration with 31-bit offsets)
    const bool small_spectra = (unsigned long long)n1 * n2 * m->SF * m->nh * sizeof(float2) < (1ULL << 31);
    if (!lp.direct && !mag && !p.nuc_ff && p.variant != 3 && m->nclass < m->S && small_spectra &&
        m->order <= kMaxOrderFast) {
        bool halves = true, whole = true;
        for (int i = 0; i < m->S; ++i) {
            const double r2 = m->frac[3 * m->site_of[i] + 1];
            const double t2 = 2.0 * r2;
            if (t2 != std::floor(t2)) halves = false;
            if (r2 != std::floor(r2)) whole = false;
            p.sgn2[i] = ((long long)std::floor(t2) % 2 == 0) ? 1 : -1;
        }
        const int L2 = whole ? 1 : 2;
        // k3 slices (variant 4: none): smaller blocks, two of them resident per CU
        const bool sliced = tb->work3 != nullptr && p.variant != 4;
        const int n3s = sliced ? tb->n3s : n3;
        const size_t bs = (size_t)m->nclass * L2 * n3s * n_pairs(m->order);
        // two planes per block: level A buffers of both, the weights of level A, then
        // the class phases
        const bool par = p.parity && p.variant != 2;
        const size_t lds = sizeof(float2) * (2 * bs + (size_t)4 * m->S * (m->order + 1) +
                                             (par ? 0 : (size_t)m->nclass * tb->nH3span));
        if (halves && lds <= 140 * 1024) {
            p.fold = 1;
            p.fold_l2 = L2;
            p.n3s = n3s;
            p.bs_elems = (int)bs;
            p.xs_elems = 0;
            p.work = sliced ? tb->work3 : tb->work2;
            p.nwork = sliced ? tb->nwork3 : tb->nwork2;
            p.k3tab = tb->k3tab;
            for (int s = 0; s < 8; ++s) p.hmin_s[s] = sliced ? tb->hmin_slice[s] : tb->hmin_all;
            lp.block = 2 * (sliced ? tb->block3 : tb->block);
            lp.lds = lds;
            // a slice covers part of each 128-byte line of a row: cached stores only
            if (sliced) p.ostream = 0;
        }
    }

    BraggParams& q = lp.bp;
    std::memset(&q, 0, sizeof(q));
    q.sums = m->d_sums; q.out = out;
    q.opitch = lay.pitch; q.ooff = lay.off;
    for (int a = 0; a < 3; ++a) {
        q.g0[a] = bx.g0[a]; q.cnt[a] = bx.cnt[a]; q.n[a] = m->n[a];
        q.Hlo[a] = (int)ceildiv_l(bx.g0[a], m->n[a]);
        const int hi = (int)floordiv_l((long)bx.g0[a] + bx.cnt[a] - 1, m->n[a]);
        q.nH[a] = std::max(0, hi - q.Hlo[a] + 1);
    }
    if (bx.half) q.nH[0] = std::max(0, std::min(q.nH[0], 1 - q.Hlo[0]));   // planes G1 <= 0
    q.S = m->S; q.T = m->T; q.M = m->M; q.kind = m->kind;
    q.scale = C / m->normN;
    q.site = m->d_site;
    if (m->kind == DSX_NUCLEAR) {
        int t = 0;
        for (int d = 0; d <= m->order; ++d)
            for (int pp = d; pp >= 0; --pp)
                for (int qq = d - pp; qq >= 0; --qq) {
                    q.mono[3 * t] = (int8_t)pp; q.mono[3 * t + 1] = (int8_t)qq; q.mono[3 * t + 2] = (int8_t)(d - pp - qq);
                    ++t;
                }
    }
    if (m->dw_order > 0) {
        int t = 0;
        for (int d = 0; d <= m->dw_order; ++d)
            for (int pp = d; pp >= 0; --pp)
                for (int qq = d - pp; qq >= 0; --qq) {
                    q.mono[3 * t] = (int8_t)pp; q.mono[3 * t + 1] = (int8_t)qq; q.mono[3 * t + 2] = (int8_t)(d - pp - qq);
                    ++t;
                }
        q.dwc = m->d_dwc;
        q.dwT = m->dwT;
    }
    for (int i = 0; i < 9; ++i) q.recip[i] = m->recip[i];
    q.has_ff = m->has_ff ? 1 : 0;
    return DSX_OK;
}

dsx_status ensure_spectra(dsx_model m, hipStream_t st, bool force = false)
{
    if (!m->dirty && !force) return DSX_OK;
    SumsParams sp{};
    sp.occ = m->has_occ ? m->d_occ : nullptr;
    sp.vec = m->d_vec;
    sp.partial = m->d_partial; sp.sums = m->d_sums;
    sp.M = m->M; sp.S = m->S; sp.ncell = m->ncell; sp.T = m->T; sp.kind = m->kind;
    sp.chunk = m->sum_chunk; sp.nchunk = m->sum_chunks;
    HIPCHK(m, timed("sums", st, [&] { return launch_sums(sp, m->order, st); }));
    if (m->dw_order > 0) {
        // the Debye-Waller factor of Eq. dw: float64 sums of the displacement monomials
        // (the partials are free again: the spins' reduction ran before on this stream)
        SumsParams dp = sp;
        dp.vec = m->d_dsp; dp.sums = m->d_dwsums; dp.T = m->dwT; dp.kind = DSX_NUCLEAR;
        HIPCHK(m, timed("dw_sums", st, [&] { return launch_sums(dp, m->dw_order, st); }));
        const DwParams dwp{m->d_dwsums, m->d_dwc, m->M, m->S, m->dwT};
        HIPCHK(m, timed("dw_mean", st, [&] { return launch_dw_mean(dwp, st); }));
    }

    PlaneParams pp;
    std::memset(&pp, 0, sizeof(pp));
    pp.occ = sp.occ; pp.vec = m->d_vec; pp.sums = m->d_sums; pp.X = m->d_X;
    pp.tw2 = m->d_tw[1]; pp.tw3 = m->d_tw[2];
    pp.p2 = m->plan[1]; pp.p3 = m->plan[2];
    pp.n1 = m->n[0]; pp.n2 = m->n[1]; pp.n3 = m->n[2]; pp.nh = m->nh;
    pp.S = m->S; pp.F = m->F; pp.T = m->T; pp.M = m->M; pp.kind = m->kind; pp.first_mono = m->first_mono;
    pp.npl = 1;
    const int npairs = (m->n[1] + 1) / 2;
    pp.buf_elems = std::max(npairs * m->n[2], m->n[1] * m->nh);
    // fields batched per block: more butterflies per pass, LDS <= 24 KB, and
    // at least ~2048 blocks when the problem allows it
    const long long planes = (long long)m->M * m->S * m->n[0];
    int fb = (int)std::max<size_t>(1, (24 * 1024 / sizeof(float2) - m->n[1] - m->n[2]) / (2 * (size_t)pp.buf_elems));
    fb = std::min(fb, 4);
    while (fb > 1 && planes * ((m->F + fb - 1) / fb) < 2048) --fb;
    if (m->tune_fchunk > 0) fb = m->tune_fchunk;
    pp.fchunk = std::min(fb, m->F);
    pp.nfchunk = (m->F + pp.fchunk - 1) / pp.fchunk;
    // a plane too large for the LDS (edges up to 256): rows along axis 3 in blocks of a
    // few row pairs, then axis 2 in place like axis 1
    const bool by_rows = planes_lds_bytes(pp) > 150 * 1024;
    if (by_rows) {
        pp.row_pairs = std::max(1, std::min(npairs, 4096 / (m->n[2] + 2)));
        pp.nrchunk = (npairs + pp.row_pairs - 1) / pp.row_pairs;
        pp.buf_elems = std::max(pp.row_pairs * m->n[2], 2 * pp.row_pairs * m->nh);
        pp.fchunk = 1;
        pp.nfchunk = m->F;
    }
    if (!by_rows) {
        // small planes: several lattice planes per block (about 1024 cells), in <= 32 KB of LDS
        int npl = std::max(1, 1024 / (m->n[1] * m->n[2] * pp.fchunk));
        npl = std::min(npl, m->n[0]);
        for (pp.npl = npl; pp.npl > 1 && planes_lds_bytes(pp) > 32 * 1024; --pp.npl) {}
    }
    if (m->kind == DSX_NUCLEAR) {
        // spectra order: pairs (q, r) by e = q + r, q descending; p ascending within
        int f = 0;
        for (int e = 0; e <= m->order; ++e)
            for (int q = e; q >= 0; --q)
                for (int p = 0; p <= m->order - e; ++p) {
                    if (p == 0 && e == 0 && m->first_mono == 1) continue;
                    pp.mono[3 * f] = (int8_t)p; pp.mono[3 * f + 1] = (int8_t)q; pp.mono[3 * f + 2] = (int8_t)(e - q);
                    ++f;
                }
    }
    HIPCHK(m, timed("fft_planes", st, [&] { return launch_fft_planes(pp, st); }));
    if (by_rows) {
        // axis 2 in place: the spectra seen as [M n1][n2][1][S F nh]
        Axis1Params a2{};
        a2.X = m->d_X; a2.tw1 = m->d_tw[1]; a2.p1 = m->plan[1];
        a2.n1 = m->n[1]; a2.n2 = 1; a2.cols = m->SF * m->nh; a2.M = m->M * m->n[0];
        a2.tc = m->n[1] <= 64 ? 64 : 32;
        a2.ncolblk = (a2.cols + a2.tc - 1) / a2.tc;
        HIPCHK(m, timed("fft_axis2", st, [&] { return launch_fft_axis1(a2, st); }));
    }

    // axis 1: for each k1 the (k2, field, k3) columns are contiguous, so they are tiled as
    // one run of n2 S F nh columns (a small box fills whole tiles instead of one per k2)
    Axis1Params ap{};
    ap.X = m->d_X; ap.tw1 = m->d_tw[0]; ap.p1 = m->plan[0];
    ap.n1 = m->n[0]; ap.n2 = m->n[1]; ap.cols = m->SF * m->nh; ap.M = m->M;
    if ((long long)ap.n2 * ap.cols <= (1LL << 30)) { ap.cols *= ap.n2; ap.n2 = 1; }
    ap.tc = m->tune_tc > 0 ? m->tune_tc : (m->n[0] <= 64 ? 64 : 32);
    ap.ncolblk = (ap.cols + ap.tc - 1) / ap.tc;
    HIPCHK(m, timed("fft_axis1", st, [&] { return launch_fft_axis1(ap, st); }));
    m->dirty = false;
    return DSX_OK;
}

dsx_status run_box(dsx_model m, const Box& bx, float* dout, const Layout& lay, hipStream_t st)
{
    LaunchPlan lp;
    dsx_status s = plan_recombine(m, bx, dout, lay, lp);
    if (s != DSX_OK) return s;
    if (lp.direct)
        HIPCHK(m, timed("recombine", st, [&] { return launch_recombine_direct(lp.rp, st); }));
    else if (lp.mag_rows)
        HIPCHK(m, timed("recombine", st, [&] { return launch_recombine_magnetic_rows(lp.rp, lp.block, lp.lds, st); }));
    else if (m->kind == DSX_MAGNETIC)
        HIPCHK(m, timed("recombine", st, [&] { return launch_recombine_magnetic(lp.rp, lp.hc, lp.block, lp.lds, st); }));
    else
        HIPCHK(m, timed("recombine", st, [&] { return launch_recombine_nuclear(lp.rp, m->order, lp.hc, lp.block, lp.lds, st); }));
    HIPCHK(m, timed("bragg", st, [&] { return launch_bragg(lp.bp, m->order, st); }));
    return DSX_OK;
}

dsx_status ready(dsx_model m)
{
    for (int c = 0; c < m->M; ++c)
        if (!m->set[c]) return fail(DSX_ERR_STATE, "configuration " + std::to_string(c) + " has no sites set");
    if (!m->grid_set) return fail(DSX_ERR_STATE, "no output grid set");
    return DSX_OK;
}

dsx_status stage(dsx_model m, size_t elems, float** p)
{
    if (m->stage_cap < elems) {
        dfree(m->d_stage);
        m->d_stage = nullptr; m->stage_cap = 0;
        hipError_t e = hipMalloc(&m->d_stage, elems * sizeof(float));
        if (e == hipErrorOutOfMemory) return fail(DSX_ERR_NOMEM, "out of device memory for the host output staging");
        HIPCHK(m, e);
        m->stage_cap = elems;
    }
    *p = m->d_stage;
    return DSX_OK;
}

}  // namespace

namespace {
dsx_status prepare_intensity(dsx_model m);
dsx_status enqueue_intensity(dsx_model m, float* dout, hipStream_t st, bool force);
}  // namespace

extern "C" {

int32_t dsx_version(void) { return 100; }

dsx_status dsx_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return DSX_OK;
}

dsx_status dsx_profile_select(const char* kernel)
{
    if (kernel && std::strlen(kernel) >= sizeof(dsx_kernel_stat{}.name))
        return fail(DSX_ERR_ARG, "kernel name longer than a dsx_kernel_stat name");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.only = kernel ? kernel : "";
    return DSX_OK;
}

static int32_t profile_read_impl(dsx_kernel_stat* out, int32_t max);

int32_t dsx_profile_read(dsx_kernel_stat* out, int32_t max)
{
    try {
        return profile_read_impl(out, max);
    } catch (...) {
        return 0;
    }
}

static int32_t profile_read_impl(dsx_kernel_stat* out, int32_t max)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto& p : g_prof.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& s = g_prof.stats[p.name];
            s.first += 1;
            s.second += ms;
        }
        g_prof.pool.push_back(p.a);
        g_prof.pool.push_back(p.b);
    }
    g_prof.pending.clear();
    int32_t i = 0;
    for (auto& kv : g_prof.stats) {
        if (out && i < max) {
            std::memset(out[i].name, 0, sizeof(out[i].name));
            std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = kv.second.first;
            out[i].total_ms = kv.second.second;
        }
        ++i;
    }
    return i;
}

dsx_status dsx_profile_reset(void)
{
    dsx_profile_read(nullptr, 0);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.stats.clear();
    return DSX_OK;
}

const char* dsx_last_error(void) { return g_err.c_str(); }

dsx_status dsx_plan_query(const dsx_model_desc* d, dsx_plan_info* info)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = validate_desc(d);
        if (s != DSX_OK) return s;
        if (!info) return fail(DSX_ERR_ARG, "info is NULL");
        const Sizes z = sizes_of(d);
        info->fields_per_site = z.F;
        info->total_fields = d->n_configs * d->n_sites * z.F;
        info->n_classes = z.nclass;
        info->reserved = 0;
        info->spectrum_bytes = z.spectrum_bytes;
        info->device_bytes = z.device_bytes;
        return DSX_OK;
    });
}

}  // extern "C"

namespace {

dsx_status create_model_body(const dsx_model_desc* d, bool transient, dsx_model m, dsx_model* out);

// Builds a model; `transient` leaves the spectra and partial-sum buffers to a server.
dsx_status create_model_impl(const dsx_model_desc* d, bool transient, dsx_model* out)
{
    dsx_status s = validate_desc(d);
    if (s != DSX_OK) return s;
    if (!out) return fail(DSX_ERR_ARG, "out is NULL");
    *out = nullptr;
    dsx_model m = new (std::nothrow) dsx_model_s();
    if (!m) return fail(DSX_ERR_NOMEM, "host allocation failed");
    dsx_status st;
    try {
        st = create_model_body(d, transient, m, out);
    } catch (...) {
        free_model(m);
        delete m;
        throw;
    }
    if (st != DSX_OK) {
        free_model(m);
        delete m;
    }
    return st;
}

// The model's description, plan and device state; on failure create_model_impl
// releases whatever it allocated.
dsx_status create_model_body(const dsx_model_desc* d, bool transient, dsx_model m, dsx_model* out)
{
    std::memcpy(m->cell, d->cell, sizeof(m->cell));
    for (int a = 0; a < 3; ++a) m->n[a] = d->n[a];
    m->S = d->n_sites; m->kind = d->kind; m->has_occ = d->has_occ ? 1 : 0;
    m->order = d->kind == DSX_NUCLEAR ? d->taylor_order : 0;
    m->M = d->n_configs;
    m->frac.assign(d->frac, d->frac + 3 * m->S);
    m->b.assign(d->b, d->b + m->S);
    // per site: the 7 form-factor parameters (f = 1 when none are given) and the
    // Debye-Waller B (0 when none is given)
    m->has_ff = d->ff != nullptr;
    if (m->has_ff) {
        m->ff.assign((size_t)8 * m->S, 0.0);
        for (int mu = 0; mu < m->S; ++mu)
            for (int k = 0; k < 7; ++k) m->ff[8 * mu + k] = d->ff[7 * mu + k];
    }
    if (d->kind == DSX_MAGNETIC && d->taylor_order > 0) {
        m->dw_order = d->taylor_order;
        m->dwT = n_monomials(m->dw_order);
    }
    reciprocal_basis(m->cell, m->recip);
    int npos = m->S;
    if (d->pos_id) {
        std::vector<int> ids(d->pos_id, d->pos_id + m->S);
        std::sort(ids.begin(), ids.end());
        npos = (int)(std::unique(ids.begin(), ids.end()) - ids.begin());
    }
    const Sizes z = sizes_of(d);
    m->ncell = z.ncell; m->nh = z.nh; m->F = z.F; m->T = z.T; m->first_mono = z.first_mono;
    m->SF = m->S * m->F;
    m->normN = d->norm_N > 0 ? d->norm_N : (double)m->ncell * npos;
    m->nclass = count_classes(d, &m->site_of, &m->class_of);
    // site chunks for the recombination's LDS budget: level-A buffer of the chunk's
    // sites plus the staging area of one site (nuclear) or of the chunk (magnetic);
    // 72 KB keeps two 512-thread blocks per CU, larger plans take up to 150 KB.
    const bool mag = m->kind == DSX_MAGNETIC;
    const size_t per_site = sizeof(float2) * (size_t)(mag ? 3 : n_pairs(m->order)) * m->n[2];
    const size_t stage_fixed = mag ? 0 : sizeof(float2) * (size_t)m->F * m->nh;
    const size_t stage_site = mag ? sizeof(float2) * 6 * (size_t)m->nh : 0;
    size_t budget = 72 * 1024;
    if (stage_fixed + per_site + stage_site > budget) budget = 150 * 1024;
    const int per_chunk = (int)std::max<size_t>(1, (budget - stage_fixed) / (per_site + stage_site));
    m->sc_start.clear();
    for (int i = 0; i < m->S; i += per_chunk) m->sc_start.push_back(i);
    m->sc_start.push_back(m->S);
    const int chunk_sites = std::min(per_chunk, m->S);
    m->bs_elems = (int)(per_site / sizeof(float2)) * chunk_sites;
    m->xs_elems = (int)((stage_fixed + stage_site * chunk_sites) / sizeof(float2));
    m->chunk_lds = per_site * chunk_sites + stage_fixed + stage_site * chunk_sites;
    for (int a = 0; a < 3; ++a) m->plan[a] = make_plan(m->n[a]);
    m->set.assign(m->M, 0);
    (void)hipGetDevice(&m->device);

    auto alloc = [&](void** p, size_t bytes) -> hipError_t { return hipMalloc(p, std::max<size_t>(bytes, 16)); };
    const size_t M = m->M, S = m->S, nc = m->ncell;
    m->sum_chunk = sums_chunk(m->ncell, (long long)m->M * m->S);
    m->sum_chunks = (m->ncell + m->sum_chunk - 1) / m->sum_chunk;
    hipError_t e = hipSuccess;
    if (m->has_occ && e == hipSuccess) e = alloc((void**)&m->d_occ, M * S * nc * sizeof(float));
    if ((m->kind == DSX_MAGNETIC || m->order > 0) && e == hipSuccess)
        e = alloc((void**)&m->d_vec, M * S * nc * 3 * sizeof(float));
    m->spectrum_bytes = (size_t)z.spectrum_bytes;
    // the partial sums serve the spins' and (after them, same stream) the displacements' sums
    m->partial_bytes = M * S * m->sum_chunks * std::max(m->T, m->dwT) * sizeof(double);
    if (e == hipSuccess && !transient) e = alloc((void**)&m->d_partial, m->partial_bytes);
    if (e == hipSuccess) e = alloc((void**)&m->d_sums, M * S * m->T * sizeof(double));
    if (m->dw_order > 0) {
        if (e == hipSuccess) e = alloc((void**)&m->d_dsp, M * S * nc * 3 * sizeof(float));
        if (e == hipSuccess) e = alloc((void**)&m->d_dwsums, M * S * m->dwT * sizeof(double));
        if (e == hipSuccess) e = alloc((void**)&m->d_dwc, S * m->dwT * sizeof(double));
    }
    if (e == hipSuccess && !transient) e = alloc((void**)&m->d_X, (size_t)z.spectrum_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->order_ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        std::vector<double> site((size_t)m->S * 12, 0.0);
        for (int mu = 0; mu < m->S; ++mu) {
            for (int a = 0; a < 3; ++a) site[12 * mu + a] = m->frac[3 * mu + a];
            site[12 * mu + 3] = m->b[mu];
            for (int k = 0; k < 8; ++k) site[12 * mu + 4 + k] = m->has_ff ? m->ff[8 * mu + k] : 0.0;
        }
        e = alloc((void**)&m->d_site, site.size() * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpy(m->d_site, site.data(), site.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    for (int a = 0; a < 3 && e == hipSuccess; ++a) {
        const int n = m->n[a];
        std::vector<float2> tw(n);
        for (int t = 0; t < n; ++t) tw[t] = cis((double)t / n);
        e = alloc((void**)&m->d_tw[a], sizeof(float2) * n);
        if (e == hipSuccess) e = hipMemcpy(m->d_tw[a], tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (e == hipErrorOutOfMemory) return fail(DSX_ERR_NOMEM, "out of device memory for the model");
        return fail(DSX_ERR_DEVICE, std::string("create_model: ") + hipGetErrorString(e));
    }
    *out = m;
    return DSX_OK;
}

// Direct compute calls own their buffers; a served model computes only through its server.
dsx_status check_direct(dsx_model m)
{
    dsx_status s = check_model(m);
    if (s != DSX_OK) return s;
    if (m->server) return fail(DSX_ERR_STATE, "the model belongs to a server: submit requests to it");
    return DSX_OK;
}

}  // namespace

extern "C" {

dsx_status dsx_create_model(const dsx_model_desc* d, dsx_model* out)
{
    return guarded([&]() -> dsx_status {
        return create_model_impl(d, false, out);
    });
}

dsx_status dsx_set_sites(dsx_model m, int32_t config, const float* occ, const float* disp,
                         const float* spin, int32_t where)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_model(m);
        if (s != DSX_OK) return s;
        if (config < 0 || config >= m->M) return fail(DSX_ERR_ARG, "config out of range");
        if (where != DSX_HOST && where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
        if (m->has_occ && !occ) return fail(DSX_ERR_ARG, "occ is required (has_occ != 0)");
        const float* vec = m->kind == DSX_MAGNETIC ? spin : disp;
        const bool need_vec = m->kind == DSX_MAGNETIC || m->order > 0;
        if (need_vec && !vec)
            return fail(DSX_ERR_ARG, m->kind == DSX_MAGNETIC ? "spin is required" : "disp is required (taylor_order > 0)");
        if (m->dw_order > 0 && !disp) return fail(DSX_ERR_ARG, "disp is required (taylor_order > 0)");
        if (m->queued.load() > 0) return fail(DSX_ERR_BUSY, "the model has requests queued at its server");
        HIPCHK(m, hipStreamSynchronize(m->last_stream));   // no pending work still reads the inputs
        const hipMemcpyKind kind = where == DSX_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        const size_t per = (size_t)m->S * m->ncell;
        if (m->has_occ) HIPCHK(m, hipMemcpy(m->d_occ + per * config, occ, per * sizeof(float), kind));
        if (need_vec) HIPCHK(m, hipMemcpy(m->d_vec + 3 * per * config, vec, 3 * per * sizeof(float), kind));
        if (m->dw_order > 0) HIPCHK(m, hipMemcpy(m->d_dsp + 3 * per * config, disp, 3 * per * sizeof(float), kind));
        if (where == DSX_DEVICE) HIPCHK(m, hipStreamSynchronize(nullptr));
        m->set[config] = 1;
        m->dirty = true;
        return DSX_OK;
    });
}

dsx_status dsx_set_sites_async(dsx_model m, int32_t config, const float* occ, const float* disp,
                               const float* spin, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_model(m);
        if (s != DSX_OK) return s;
        if (config < 0 || config >= m->M) return fail(DSX_ERR_ARG, "config out of range");
        if (m->has_occ && !occ) return fail(DSX_ERR_ARG, "occ is required (has_occ != 0)");
        const float* vec = m->kind == DSX_MAGNETIC ? spin : disp;
        const bool need_vec = m->kind == DSX_MAGNETIC || m->order > 0;
        if (need_vec && !vec)
            return fail(DSX_ERR_ARG, m->kind == DSX_MAGNETIC ? "spin is required" : "disp is required (taylor_order > 0)");
        if (m->dw_order > 0 && !disp) return fail(DSX_ERR_ARG, "disp is required (taylor_order > 0)");
        if (m->server) return fail(DSX_ERR_STATE, "the model belongs to a server: its requests carry the sites");
        hipStream_t st = (hipStream_t)hip_stream;
        if ((s = follow(m, st)) != DSX_OK) return s;     // after every earlier use of the inputs
        const size_t per = (size_t)m->S * m->ncell;
        if (m->has_occ)
            HIPCHK(m, hipMemcpyAsync(m->d_occ + per * config, occ, per * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (need_vec)
            HIPCHK(m, hipMemcpyAsync(m->d_vec + 3 * per * config, vec, 3 * per * sizeof(float), hipMemcpyDeviceToDevice, st));
        if (m->dw_order > 0)
            HIPCHK(m, hipMemcpyAsync(m->d_dsp + 3 * per * config, disp, 3 * per * sizeof(float), hipMemcpyDeviceToDevice, st));
        m->set[config] = 1;
        m->dirty = true;
        return DSX_OK;
    });
}

dsx_status dsx_set_grid(dsx_model m, const int32_t g0[3], const int32_t count[3])
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_model(m);
        if (s != DSX_OK) return s;
        if (!g0 || !count) return fail(DSX_ERR_ARG, "g0 and count are required");
        if (m->pins) return fail(DSX_ERR_BUSY, "the model is recorded in a batch; destroy the batch first");
        if (m->queued.load() > 0) return fail(DSX_ERR_BUSY, "the model has requests queued at its server");
        Box bx;
        long long vox = 1;
        for (int a = 0; a < 3; ++a) {
            if (count[a] < 1) return fail(DSX_ERR_ARG, "count must be >= 1 on every axis");
            if (std::llabs((long long)g0[a]) > (1LL << 24) || count[a] > (1 << 24))
                return fail(DSX_ERR_UNSUPPORTED, "box coordinates too large");
            bx.g0[a] = g0[a]; bx.cnt[a] = count[a];
            vox *= count[a];
        }
        if (vox > (1LL << 34)) return fail(DSX_ERR_UNSUPPORTED, "box too large");
        m->box = bx;
        m->grid_set = true;
        // prepare the box's phase tables now, so that a compute call that may not allocate
        // finds them; a box the recombination cannot take is still reported by the compute
        // calls, as before
        DeviceTables* tb = nullptr;
        if (tables_for(m, bx, &tb) != DSX_OK) {
            if (m->failed) return DSX_ERR_DEVICE;
            g_err.clear();
        }
        return DSX_OK;
    });
}

dsx_status dsx_compute_intensity(dsx_model m, float* out, int32_t where, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!out) return fail(DSX_ERR_ARG, "out is NULL");
        if (where != DSX_HOST && where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
        if ((s = ready(m)) != DSX_OK) return s;
        hipStream_t st = (hipStream_t)hip_stream;
        const size_t vox = (size_t)m->box.cnt[0] * m->box.cnt[1] * m->box.cnt[2];
        float* dout = out;
        if (where == DSX_HOST && (s = stage(m, vox, &dout)) != DSX_OK) return s;
        if ((s = prepare_intensity(m)) != DSX_OK) return s;
        if ((s = follow(m, st)) != DSX_OK) return s;
        if ((s = enqueue_intensity(m, dout, st, false)) != DSX_OK) return s;
        if (where == DSX_HOST) {
            HIPCHK(m, hipMemcpyAsync(out, dout, vox * sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(m, hipStreamSynchronize(st));
        }
        return DSX_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------- no allocation
// Device scratch of dsx_compute_intensity_noalloc: the spectra and the partial lattice
// sums of one call.  Every device the library runs on holds its own copy until the
// process ends; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in there).
static __device__ __align__(256) unsigned char scratch[DSX_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_at;   // device -> its copy of `scratch`

dsx_status scratch_on(int dev, unsigned char** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_at.find(dev);
    if (it == g_scratch_at.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DSX_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        it = g_scratch_at.emplace(dev, static_cast<unsigned char*>(p)).first;
    }
    *out = it->second;
    return DSX_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

dsx_status dsx_compute_intensity_noalloc(dsx_model m, float* out, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!out) return fail(DSX_ERR_ARG, "out is NULL");
        if ((s = ready(m)) != DSX_OK) return s;
        int dev = -1;
        HIPCHK(m, hipGetDevice(&dev));
        if (dev != m->device) return fail(DSX_ERR_ARG, "the current device is not the model's device");
        const size_t xb = round256(m->spectrum_bytes), pb = round256(m->partial_bytes);
        if (xb + pb > (size_t)DSX_NOALLOC_SCRATCH_BYTES)
            return fail(DSX_ERR_UNSUPPORTED, "spectra and partial sums (" + std::to_string(xb + pb) +
                                             " bytes) exceed the " + std::to_string(DSX_NOALLOC_SCRATCH_BYTES) +
                                             "-byte scratch of dsx_compute_intensity_noalloc");
        if (!m->tables.count(m->box))
            return fail(DSX_ERR_STATE, "the grid's phase tables are not resident: dsx_set_grid prepares them "
                                       "(dsx_compute_intensity reports why it could not)");
        unsigned char* base = nullptr;
        if ((s = scratch_on(dev, &base)) != DSX_OK) return s;
        hipStream_t st = (hipStream_t)hip_stream;
        if ((s = follow(m, st)) != DSX_OK) return s;
        // the whole chain reads and writes the scratch in place of the model's own spectra
        // and partial sums; every element is written before it is read
        float2* own_x = m->d_X;
        double* own_p = m->d_partial;
        m->d_X = reinterpret_cast<float2*>(base);
        m->d_partial = reinterpret_cast<double*>(base + xb);
        s = enqueue_intensity(m, out, st, true);
        m->d_X = own_x;
        m->d_partial = own_p;
        m->dirty = true;     // the model's own spectra were not refreshed
        return s;
    });
}

}  // extern "C"

namespace {

Box grown_box(const Box& b, int mm)
{
    // grown box [g0 - m, g0 + count + m): the window of output Q_a = g0_a + i/s spans
    // G_a in [floor(Q_a) - m + 1, floor(Q_a) + m]; growing by m on both sides (one
    // unused plane below) keeps a box symmetric about 0 symmetric.
    Box ext;
    for (int a = 0; a < 3; ++a) {
        ext.g0[a] = b.g0[a] - mm;
        ext.cnt[a] = b.cnt[a] + 2 * mm;
    }
    return ext;
}

// The box the filter reads: the output box grown by the window, stored as its half
// G1 <= 0 when it is symmetric about G = 0.
Box filter_box(const Box& b, int mm)
{
    Box e = grown_box(b, mm);
    e.half = symmetric_box(e) ? 1 : 0;
    return e;
}

// Rows of the grown box start on 128-byte lines (pitch a multiple of 32 floats):
// the recombination writes each H3 step of a row as whole lines, and the filter,
// whose window points start at eoff = 1, cuts its column tiles at multiples of 64
// in window (input) coordinates, so its tiles read whole lines too.
constexpr int kExtEoff = 1;
Layout ext_layout(const Box& ext)
{
    return Layout{(ext.cnt[2] + 31) / 32 * 32, 0};
}

size_t ext_elems(const Box& ext) { return (size_t)stored_planes(ext) * ext.cnt[1] * ext_layout(ext).pitch; }

// Everything the filter needs that allocates or uploads (never inside a capture).
// lm = m of the filter, mp = m' of its cutoff modification (2: none); the window's
// half-width is lm mp / 2.
dsx_status prepare_filter(dsx_model m, int lm, int sv, int mp = 2)
{
    const int mm = lm * mp / 2;
    const Box ext = filter_box(m->box, mm);
    const size_t ext_vox = ext_elems(ext);
    if (m->ext_cap < ext_vox) {
        if (m->pins) return fail(DSX_ERR_BUSY, "the grown box would outgrow a buffer a batch has recorded");
        dfree(m->d_ext);
        m->d_ext = nullptr; m->ext_cap = 0;
        hipError_t e = hipMalloc(&m->d_ext, ext_vox * sizeof(float));
        if (e == hipErrorOutOfMemory) return fail(DSX_ERR_NOMEM, "out of device memory for the grown box");
        HIPCHK(m, e);
        m->ext_cap = ext_vox;
    }
    // normalised weights [s][2 mm]; r_cut = (1 - 1/m)/m' (Sec. V.B; m' = 2: (1 - 1/m)/2)
    const auto key = std::make_tuple(lm, mp, sv);
    if (!m->lanczos_w.count(key)) {
        const double rcut = (1.0 - 1.0 / lm) / mp;
        auto sinc = [](double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; };
        std::vector<float> w((size_t)sv * 2 * mm);
        for (int j = 0; j < sv; ++j) {
            std::vector<double> v(2 * mm);
            double tot = 0.0;
            for (int d = 0; d < 2 * mm; ++d) {
                const double dl = (double)j / sv + mm - 1 - d;
                v[d] = std::fabs(dl) < mm ? sinc(2 * M_PI * rcut * dl) * sinc(M_PI * dl / mm) : 0.0;
                tot += v[d];
            }
            for (int d = 0; d < 2 * mm; ++d) w[(size_t)j * 2 * mm + d] = (float)(v[d] / tot);
        }
        float* dw = nullptr;
        HIPCHK(m, hipMalloc(&dw, w.size() * sizeof(float)));
        HIPCHK(m, hipMemcpy(dw, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
        try {
            m->lanczos_w[key] = dw;
        } catch (...) {
            dfree(dw);
            throw;
        }
    }
    DeviceTables* tb = nullptr;
    return tables_for(m, ext, &tb);
}

dsx_status prepare_intensity(dsx_model m)
{
    DeviceTables* tb = nullptr;
    return tables_for(m, m->box, &tb);
}

// Stream-ordered launches only: spectra (when stale or forced), recombination on
// the grown box, Bragg points, filter.
dsx_status enqueue_filter(dsx_model m, int lm, int sv, float* dout, hipStream_t st, bool force, int mp = 2)
{
    dsx_status s;
    const int mm = lm * mp / 2;
    const Box ext = filter_box(m->box, mm);
    if ((s = ensure_spectra(m, st, force)) != DSX_OK) return s;
    const Layout el = ext_layout(ext);
    if ((s = run_box(m, ext, m->d_ext, el, st)) != DSX_OK) return s;
    LanczosParams lp{};
    lp.in = m->d_ext; lp.out = dout; lp.wn = m->lanczos_w[std::make_tuple(lm, mp, sv)];
    lp.ipitch = el.pitch; lp.ioff = el.off;
    lp.ihalf = stored_planes(ext);
    for (int a = 0; a < 3; ++a) { lp.e[a] = ext.cnt[a]; lp.o[a] = sv * m->box.cnt[a]; }
    lp.m = mm; lp.s = sv;
    lp.eoff = kExtEoff;
    lp.t3 = 64; lp.t1 = m->tune_lanczos_t1;
    lp.t2 = 32;
    while (lp.t2 > 1 && lanczos_lds_bytes(lp) > 150 * 1024) lp.t2 /= 2;
    while (lp.t3 > 8 && lanczos_lds_bytes(lp) > 150 * 1024) lp.t3 /= 2;
    // s = 1 on a symmetric box: compute the planes G1 <= 0 and write each also at -G
    lp.ohalf = (sv == 1 && symmetric_box(m->box)) ? (lp.o[0] + 1) / 2 : 0;
    lp.nb1 = (lp.o[0] + lp.t1 - 1) / lp.t1;
    lp.nb2 = (lp.o[1] + lp.t2 - 1) / lp.t2;
    lp.nb3 = (lp.o[2] + lp.t3 - 1) / lp.t3;
    HIPCHK(m, timed("lanczos", st, [&] { return launch_lanczos(lp, st); }));
    return DSX_OK;
}

dsx_status enqueue_intensity(dsx_model m, float* dout, hipStream_t st, bool force)
{
    dsx_status s;
    if ((s = ensure_spectra(m, st, force)) != DSX_OK) return s;
    return run_box(m, m->box, dout, dense_layout(m->box), st);
}

dsx_status check_filter_args(int32_t lanczos_m, int32_t oversample)
{
    if (lanczos_m < 2) return fail(DSX_ERR_ARG, "lanczos_m must be >= 2");
    if (oversample < 1) return fail(DSX_ERR_ARG, "oversample must be >= 1");
    if (lanczos_m > 16 || oversample > 16) return fail(DSX_ERR_UNSUPPORTED, "lanczos_m and oversample are limited to 16");
    return DSX_OK;
}

}  // namespace

extern "C" {

dsx_status dsx_noise_filter(dsx_model m, int32_t lanczos_m, int32_t oversample, float* out,
                            int32_t where, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!out) return fail(DSX_ERR_ARG, "out is NULL");
        if (where != DSX_HOST && where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
        if ((s = check_filter_args(lanczos_m, oversample)) != DSX_OK) return s;
        if ((s = ready(m)) != DSX_OK) return s;
        hipStream_t st = (hipStream_t)hip_stream;
        const size_t out_vox = (size_t)oversample * m->box.cnt[0] * oversample * m->box.cnt[1] *
                               oversample * m->box.cnt[2];
        if ((s = prepare_filter(m, lanczos_m, oversample)) != DSX_OK) return s;
        float* dout = out;
        if (where == DSX_HOST && (s = stage(m, out_vox, &dout)) != DSX_OK) return s;
        if ((s = follow(m, st)) != DSX_OK) return s;
        if ((s = enqueue_filter(m, lanczos_m, oversample, dout, st, false)) != DSX_OK) return s;
        if (where == DSX_HOST) {
            HIPCHK(m, hipMemcpyAsync(out, dout, out_vox * sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(m, hipStreamSynchronize(st));
        }
        return DSX_OK;
    });
}

dsx_status dsx_split_sites(const int32_t n[3], int32_t n_sites, const double* frac, const double* b,
                           int32_t n_configs, const float* occ, const float* disp, double tol,
                           int32_t max_sites, int32_t* n_split, double* frac_out, double* b_out,
                           int32_t* parent_out, float* occ_out)
{
    return guarded([&]() -> dsx_status {
        if (!n || !frac || !b || !disp || !n_split || !frac_out || !b_out || !parent_out || !occ_out)
            return fail(DSX_ERR_ARG, "null argument");
        for (int a = 0; a < 3; ++a)
            if (n[a] < 1 || n[a] > DSX_MAX_N) return fail(DSX_ERR_ARG, "n out of range");
        if (n_sites < 1 || n_sites > DSX_MAX_SITES || n_configs < 1 || !(tol >= 0.0))
            return fail(DSX_ERR_ARG, "bad n_sites, n_configs or tol");
        if (max_sites < 1 || max_sites > DSX_MAX_SITES) return fail(DSX_ERR_ARG, "max_sites out of range");
        const size_t ncell = (size_t)n[0] * n[1] * n[2];
        // distinct displacements per site, in the order first met; cls[c][mu][cell] = index
        std::vector<std::vector<std::array<float, 3>>> vals(n_sites);
        std::vector<int32_t> cls((size_t)n_configs * n_sites * ncell);
        int total = 0;
        for (int c = 0; c < n_configs; ++c)
            for (int mu = 0; mu < n_sites; ++mu) {
                const float* u = disp + ((size_t)c * n_sites + mu) * ncell * 3;
                auto& vs = vals[mu];
                for (size_t r = 0; r < ncell; ++r) {
                    const float* ur = u + 3 * r;
                    int k = -1;
                    for (size_t j = 0; j < vs.size() && k < 0; ++j)
                        if (std::fabs((double)ur[0] - vs[j][0]) <= tol && std::fabs((double)ur[1] - vs[j][1]) <= tol &&
                            std::fabs((double)ur[2] - vs[j][2]) <= tol)
                            k = (int)j;
                    if (k < 0) {
                        if (++total > max_sites)
                            return fail(DSX_ERR_UNSUPPORTED, "more split sites than max_sites");
                        vs.push_back({ur[0], ur[1], ur[2]});
                        k = (int)vs.size() - 1;
                    }
                    cls[((size_t)c * n_sites + mu) * ncell + r] = k;
                }
            }
        // split sites: site mu's values in order, sites in order
        std::vector<int> first(n_sites + 1, 0);
        for (int mu = 0; mu < n_sites; ++mu) first[mu + 1] = first[mu] + (int)vals[mu].size();
        for (int mu = 0; mu < n_sites; ++mu)
            for (size_t k = 0; k < vals[mu].size(); ++k) {
                const int sidx = first[mu] + (int)k;
                for (int a = 0; a < 3; ++a) frac_out[3 * sidx + a] = frac[3 * mu + a] + (double)vals[mu][k][a];
                b_out[sidx] = b[mu];
                parent_out[sidx] = mu;
            }
        const int ns = first[n_sites];
        for (int c = 0; c < n_configs; ++c)
            for (int mu = 0; mu < n_sites; ++mu) {
                const float* dl = occ ? occ + ((size_t)c * n_sites + mu) * ncell : nullptr;
                const int32_t* kk = cls.data() + ((size_t)c * n_sites + mu) * ncell;
                for (size_t k = 0; k < vals[mu].size(); ++k) {
                    float* o = occ_out + ((size_t)c * max_sites + first[mu] + k) * ncell;
                    for (size_t r = 0; r < ncell; ++r) o[r] = kk[r] == (int)k ? (dl ? dl[r] : 1.f) : 0.f;
                }
            }
        *n_split = ns;
        return DSX_OK;
    });
}

dsx_status dsx_noise_filter_spherical(dsx_model m, int32_t lanczos_m, int32_t oversample, float* out,
                                     int32_t where, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!out) return fail(DSX_ERR_ARG, "out is NULL");
        if (where != DSX_HOST && where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
        if ((s = check_filter_args(lanczos_m, oversample)) != DSX_OK) return s;
        if (lanczos_m > 4 || oversample > 4)
            return fail(DSX_ERR_UNSUPPORTED, "the spherical cutoff supports lanczos_m <= 4 and oversample <= 4");
        if ((s = ready(m)) != DSX_OK) return s;
        hipStream_t st = (hipStream_t)hip_stream;
        const int lm = lanczos_m, sv = oversample;
        const size_t out_vox = (size_t)sv * m->box.cnt[0] * sv * m->box.cnt[1] * sv * m->box.cnt[2];
        // the grown box and its tables (as for the separable filter)
        if ((s = prepare_filter(m, lm, sv)) != DSX_OK) return s;
        // weights [s^3][(2m)^3]: W_r(|Q - G|) L(Q - G), normalised per output phase
        const auto key = std::make_tuple(lm, 0, sv);
        if (!m->lanczos_w.count(key)) {
            double rmax = 1e300;
            for (int a = 0; a < 3; ++a) {
                const double len = std::sqrt(m->recip[3 * a] * m->recip[3 * a] + m->recip[3 * a + 1] * m->recip[3 * a + 1] +
                                             m->recip[3 * a + 2] * m->recip[3 * a + 2]);
                rmax = std::min(rmax, m->n[a] * M_PI / len);
            }
            const double rc = (1.0 - 1.0 / lm) * rmax;
            auto sinc = [](double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; };
            auto ball = [](double x) {
                const double ax = std::fabs(x);
                if (ax < 1e-2) return 1.0 / 3.0 - x * x / 30.0 + x * x * x * x / 840.0;
                return (std::sin(ax) - ax * std::cos(ax)) / (ax * ax * ax);
            };
            const int T = 2 * lm;
            std::vector<float> w((size_t)sv * sv * sv * T * T * T);
            std::vector<double> v((size_t)T * T * T);
            for (int j1 = 0; j1 < sv; ++j1)
            for (int j2 = 0; j2 < sv; ++j2)
            for (int j3 = 0; j3 < sv; ++j3) {
                double tot = 0.0;
                const int jj[3] = {j1, j2, j3};
                for (int t1 = 0; t1 < T; ++t1)
                for (int t2 = 0; t2 < T; ++t2)
                for (int t3 = 0; t3 < T; ++t3) {
                    const int tt[3] = {t1, t2, t3};
                    double d[3], L = 1.0, q[3] = {0.0, 0.0, 0.0};
                    for (int a = 0; a < 3; ++a) {
                        d[a] = (double)jj[a] / sv + lm - 1 - tt[a];      // Q_a - G_a
                        L *= std::fabs(d[a]) < lm ? sinc(M_PI * d[a] / lm) : 0.0;
                        for (int c = 0; c < 3; ++c) q[c] += d[a] / m->n[a] * m->recip[3 * a + c];
                    }
                    const double x = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) * rc;
                    const double wv = ball(x) * L;
                    v[((size_t)t1 * T + t2) * T + t3] = wv;
                    tot += wv;
                }
                const size_t ph = ((size_t)j1 * sv + j2) * sv + j3;
                for (size_t t = 0; t < v.size(); ++t) w[ph * v.size() + t] = (float)(v[t] / tot);
            }
            float* dw = nullptr;
            HIPCHK(m, hipMalloc(&dw, w.size() * sizeof(float)));
            HIPCHK(m, hipMemcpy(dw, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
            try {
                m->lanczos_w[key] = dw;
            } catch (...) {
                dfree(dw);
                throw;
            }
        }
        float* dout = out;
        if (where == DSX_HOST && (s = stage(m, out_vox, &dout)) != DSX_OK) return s;
        if ((s = follow(m, st)) != DSX_OK) return s;
        const Box ext = filter_box(m->box, lm);
        if ((s = ensure_spectra(m, st, false)) != DSX_OK) return s;
        const Layout el = ext_layout(ext);
        if ((s = run_box(m, ext, m->d_ext, el, st)) != DSX_OK) return s;
        LanczosParams lp{};
        lp.in = m->d_ext; lp.out = dout; lp.wn = m->lanczos_w[key];
        lp.ipitch = el.pitch; lp.ioff = el.off;
        lp.ihalf = stored_planes(ext);
        for (int a = 0; a < 3; ++a) { lp.e[a] = ext.cnt[a]; lp.o[a] = sv * m->box.cnt[a]; }
        lp.m = lm; lp.s = sv;
        lp.eoff = kExtEoff;
        HIPCHK(m, timed("lanczos_spherical", st, [&] { return launch_lanczos_stencil(lp, st); }));
        if (where == DSX_HOST) {
            HIPCHK(m, hipMemcpyAsync(out, dout, out_vox * sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(m, hipStreamSynchronize(st));
        }
        return DSX_OK;
    });
}

dsx_status dsx_noise_filter_cutoff(dsx_model m, int32_t lanczos_m, int32_t mprime, int32_t oversample,
                                   float* out, int32_t where, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!out) return fail(DSX_ERR_ARG, "out is NULL");
        if (where != DSX_HOST && where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
        if (mprime < 2 || (lanczos_m * mprime) % 2 != 0)
            return fail(DSX_ERR_ARG, "mprime must be >= 2 with lanczos_m * mprime even");
        if ((s = check_filter_args(lanczos_m, oversample)) != DSX_OK) return s;
        if (lanczos_m * mprime / 2 > 16) return fail(DSX_ERR_UNSUPPORTED, "the window half-width m m'/2 is limited to 16");
        if ((s = ready(m)) != DSX_OK) return s;
        hipStream_t st = (hipStream_t)hip_stream;
        const size_t out_vox = (size_t)oversample * m->box.cnt[0] * oversample * m->box.cnt[1] *
                               oversample * m->box.cnt[2];
        if ((s = prepare_filter(m, lanczos_m, oversample, mprime)) != DSX_OK) return s;
        float* dout = out;
        if (where == DSX_HOST && (s = stage(m, out_vox, &dout)) != DSX_OK) return s;
        if ((s = follow(m, st)) != DSX_OK) return s;
        if ((s = enqueue_filter(m, lanczos_m, oversample, dout, st, false, mprime)) != DSX_OK) return s;
        if (where == DSX_HOST) {
            HIPCHK(m, hipMemcpyAsync(out, dout, out_vox * sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(m, hipStreamSynchronize(st));
        }
        return DSX_OK;
    });
}

dsx_status dsx_filter_points(dsx_model m, int32_t lanczos_m, int32_t mprime, int64_t npts, const double* q,
                             float* out, int32_t where, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (npts < 0 || (npts > 0 && (!q || !out))) return fail(DSX_ERR_ARG, "bad point list");
        if (where != DSX_HOST && where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
        if (lanczos_m < 2 || mprime < 2 || (lanczos_m * mprime) % 2 != 0)
            return fail(DSX_ERR_ARG, "need lanczos_m >= 2, mprime >= 2 and lanczos_m * mprime even");
        const int w = lanczos_m * mprime / 2;
        if (w > kPointsMaxHalfwidth) return fail(DSX_ERR_UNSUPPORTED, "the window half-width m m'/2 is limited to 8 here");
        if ((s = ready(m)) != DSX_OK) return s;
        if (npts == 0) return DSX_OK;
        // the box of every window: floor(Q_a) - w + 1 .. floor(Q_a) + w
        long lo[3] = {LONG_MAX, LONG_MAX, LONG_MAX}, hi[3] = {LONG_MIN, LONG_MIN, LONG_MIN};
        for (int64_t i = 0; i < npts; ++i)
            for (int a = 0; a < 3; ++a) {
                const double v = q[3 * i + a];
                if (!std::isfinite(v) || std::fabs(v) > 1e6) return fail(DSX_ERR_ARG, "points must be finite, |Q| <= 1e6");
                const long f = (long)std::floor(v);
                lo[a] = std::min(lo[a], f - w + 1);
                hi[a] = std::max(hi[a], f + w);
            }
        // a box nearly symmetric about G = 0 is made symmetric (at most ~10 % more volume):
        // the recombination then evaluates half of it (I(-G) = I(G))
        bool near_sym = true;
        for (int a = 0; a < 3; ++a) {
            const long r = std::max(std::labs(lo[a]), std::labs(hi[a]));
            if ((double)(2 * r + 1) > 1.1 * (double)(hi[a] - lo[a] + 1) + 2.0) near_sym = false;
        }
        if (near_sym)
            for (int a = 0; a < 3; ++a) {
                const long r = std::max(std::labs(lo[a]), std::labs(hi[a]));
                lo[a] = -r; hi[a] = r;
            }
        Box bx;
        for (int a = 0; a < 3; ++a) { bx.g0[a] = (int)lo[a]; bx.cnt[a] = (int)(hi[a] - lo[a] + 1); }
        const size_t vox = (size_t)bx.cnt[0] * bx.cnt[1] * bx.cnt[2];
        DeviceTables* tb = nullptr;
        if ((s = tables_for(m, bx, &tb)) != DSX_OK) return s;
        if (m->pts_cap < vox || m->q_cap < (size_t)npts) {
            if (m->pins) return fail(DSX_ERR_BUSY, "a batch has recorded this model's buffers");
        }
        if (m->pts_cap < vox) {
            dfree(m->d_pts); m->d_pts = nullptr; m->pts_cap = 0;
            hipError_t e = hipMalloc(&m->d_pts, vox * sizeof(float));
            if (e == hipErrorOutOfMemory) return fail(DSX_ERR_NOMEM, "out of device memory for the points' box");
            HIPCHK(m, e);
            m->pts_cap = vox;
        }
        if (m->q_cap < (size_t)npts) {
            dfree(m->d_q); m->d_q = nullptr; m->q_cap = 0;
            hipError_t e = hipMalloc(&m->d_q, (size_t)npts * 3 * sizeof(double));
            if (e == hipErrorOutOfMemory) return fail(DSX_ERR_NOMEM, "out of device memory for the points");
            HIPCHK(m, e);
            m->q_cap = (size_t)npts;
        }
        hipStream_t st = (hipStream_t)hip_stream;
        float* dout = out;
        if (where == DSX_HOST && (s = stage(m, (size_t)npts, &dout)) != DSX_OK) return s;
        if ((s = follow(m, st)) != DSX_OK) return s;
        HIPCHK(m, hipMemcpyAsync(m->d_q, q, (size_t)npts * 3 * sizeof(double), hipMemcpyHostToDevice, st));
        if ((s = ensure_spectra(m, st, false)) != DSX_OK) return s;
        if ((s = run_box(m, bx, m->d_pts, dense_layout(bx), st)) != DSX_OK) return s;
        PointsParams pp{};
        pp.in = m->d_pts; pp.q = m->d_q; pp.out = dout; pp.npts = npts;
        for (int a = 0; a < 3; ++a) { pp.e0[a] = bx.g0[a]; pp.e[a] = bx.cnt[a]; }
        pp.w = w;
        pp.rcut = (float)((1.0 - 1.0 / lanczos_m) / mprime);
        HIPCHK(m, timed("lanczos_points", st, [&] { return launch_lanczos_points(pp, st); }));
        if (where == DSX_HOST) {
            HIPCHK(m, hipMemcpyAsync(out, dout, (size_t)npts * sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(m, hipStreamSynchronize(st));
        } else {
            // the point list is a host array read by the copy above: wait before returning
            HIPCHK(m, hipStreamSynchronize(st));
        }
        return DSX_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------- autotuner
namespace {

std::string tune_key(dsx_model m, int lm)
{
    std::ostringstream k;
    k << "gfx950|" << m->kind << "|" << m->n[0] << "," << m->n[1] << "," << m->n[2] << "|S" << m->S
      << "|N" << m->order << "|M" << m->M << "|occ" << m->has_occ << "|box" << m->box.g0[0] << ","
      << m->box.g0[1] << "," << m->box.g0[2] << "," << m->box.cnt[0] << "," << m->box.cnt[1] << ","
      << m->box.cnt[2] << "|m" << lm;
    return k.str();
}

std::mutex g_tune_mu;

struct FftChoice {
    int tc = 0;
    std::string plan[3];   // empty: default
};

bool tune_lookup(const std::string& key, int* v, int* fc, int* t1, FftChoice* fft)
{
    const char* path = std::getenv("DSX_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.substr(0, tab) != key) continue;
        std::istringstream in(line.substr(tab + 1));
        int a, b, c;
        if (in >> a >> b >> c) {
            *v = a; *fc = b; *t1 = c; found = true;
            // optional: axis-1 column tile and the three radix sequences
            FftChoice f;
            if (in >> f.tc >> f.plan[0] >> f.plan[1] >> f.plan[2]) *fft = f;
            else *fft = FftChoice{};
        }
    }
    return found;
}

void tune_store(const std::string& key, int v, int fc, int t1, const FftChoice& fft)
{
    const char* path = std::getenv("DSX_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ofstream f(path, std::ios::app);
    f << key << "\t" << v << " " << fc << " " << t1 << " " << fft.tc << " " << fft.plan[0] << " " << fft.plan[1]
      << " " << fft.plan[2] << "\n";
}

// Minimum over `reps` timed runs of fn() on stream st (milliseconds), or < 0 on error.
template <typename Fn>
float time_min(hipStream_t st, int reps, Fn fn)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.f;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return -1.f; }
    float best = -1.f;
    for (int r = 0; r < reps; ++r) {
        if (hipEventRecord(a, st) != hipSuccess) break;
        if (fn() != DSX_OK) { best = -1.f; break; }
        if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) break;
        if (best < 0.f || ms < best) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

}  // namespace

extern "C" {

dsx_status dsx_autotune(dsx_model m, int32_t lanczos_m, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if ((s = ready(m)) != DSX_OK) return s;
        const bool filt = lanczos_m >= 2;
        if (lanczos_m != 0 && (s = check_filter_args(lanczos_m, 1)) != DSX_OK) return s;
        hipStream_t st = (hipStream_t)hip_stream;
        const std::string key = tune_key(m, lanczos_m);
        int v = 0, fc = 0, t1 = 12;
        FftChoice fch;
        if (tune_lookup(key, &v, &fc, &t1, &fch)) {
            m->tune_recomb_variant = v; m->tune_fchunk = fc; m->tune_lanczos_t1 = t1;
            if (fch.tc == 0 || fch.tc == 16 || fch.tc == 32 || fch.tc == 64) m->tune_tc = fch.tc;
            for (int a = 0; a < 3; ++a) {
                AxisPlan p{};
                if (!fch.plan[a].empty() && parse_plan(fch.plan[a], m->n[a], &p)) m->plan[a] = p;
            }
            m->dirty = true;
            m->tuned = true;
            return DSX_OK;
        }
        if ((s = prepare_intensity(m)) != DSX_OK) return s;
        if (filt && (s = prepare_filter(m, lanczos_m, 1)) != DSX_OK) return s;
        float* scratch = nullptr;
        const size_t vox = (size_t)m->box.cnt[0] * m->box.cnt[1] * m->box.cnt[2];
        if ((s = stage(m, vox, &scratch)) != DSX_OK) return s;
        if ((s = follow(m, st)) != DSX_OK) return s;
        const bool prof = g_prof.on;
        g_prof.on = false;
        // FFT: fields per plane block
        float best = -1.f;
        int best_fc = 0;
        for (int cand : {0, 1, 2, 4}) {
            m->tune_fchunk = cand;
            const float t = time_min(st, 3, [&] { return ensure_spectra(m, st, true); });
            if (t >= 0.f && (best < 0.f || t < best)) { best = t; best_fc = cand; }
        }
        m->tune_fchunk = best_fc;
        // FFT radix orders of the axes the LDS kernels transform (the register kernels of
        // edges 8, 16, 32 have a fixed order), one axis at a time
        const auto reg = [](int n) { return n == 8 || n == 16 || n == 32; };
        for (int a : {2, 1, 0}) {
            const bool used = a == 0 ? !reg(m->n[0]) : !(reg(m->n[1]) && reg(m->n[2]));
            if (!used) continue;
            const std::vector<AxisPlan> cands = plan_candidates(m->n[a], 12);
            if (cands.size() < 2) continue;
            best = -1.f;
            AxisPlan bestp = m->plan[a];
            for (const AxisPlan& c : cands) {
                m->plan[a] = c;
                const float t = time_min(st, 3, [&] { return ensure_spectra(m, st, true); });
                if (t >= 0.f && (best < 0.f || t < best)) { best = t; bestp = c; }
            }
            m->plan[a] = bestp;
        }
        // columns per block of the LDS axis-1 FFT
        if (!reg(m->n[0])) {
            best = -1.f;
            int best_tc = 0;
            for (int cand : {16, 32, 64}) {
                if (sizeof(float2) * (size_t)m->n[0] * (1 + 2 * (size_t)cand) > 160 * 1024) continue;
                m->tune_tc = cand;
                const float t = time_min(st, 3, [&] { return ensure_spectra(m, st, true); });
                if (t >= 0.f && (best < 0.f || t < best)) { best = t; best_tc = cand; }
            }
            m->tune_tc = best_tc;
        }
        // recombination form (the parity form only exists for nuclear models whose r3 are halves)
        best = -1.f;
        int best_v = 0;
        const Box b = filt ? filter_box(m->box, lanczos_m) : m->box;
        float* dst = filt ? m->d_ext : scratch;
        for (int cand : {0, 2, 3, 4, 5}) {
            if (cand != 0 && m->kind != DSX_NUCLEAR) continue;
            if (cand == 5 && !direct_form_applies(m)) continue;
            m->tune_recomb_variant = cand;
            const Layout lay = filt ? ext_layout(b) : dense_layout(b);
            const float t = time_min(st, 3, [&] { return run_box(m, b, dst, lay, st); });
            if (t >= 0.f && (best < 0.f || t < best)) { best = t; best_v = cand; }
        }
        m->tune_recomb_variant = best_v;
        // filter: planes per block
        int best_t1 = 12;
        if (filt) {
            best = -1.f;
            for (int cand : {4, 6, 8, 12, 16, 20, 26, 32, 52, 64}) {
                m->tune_lanczos_t1 = cand;
                const float t = time_min(st, 3, [&] { return enqueue_filter(m, lanczos_m, 1, scratch, st, false); });
                if (t >= 0.f && (best < 0.f || t < best)) { best = t; best_t1 = cand; }
            }
            m->tune_lanczos_t1 = best_t1;
        }
        g_prof.on = prof;
        if (m->failed) return fail(DSX_ERR_DEVICE, "device error during tuning");
        m->tuned = true;
        m->dirty = true;      // the spectra of the last candidate: recomputed with the chosen plans
        FftChoice chosen;
        chosen.tc = m->tune_tc;
        for (int a = 0; a < 3; ++a) chosen.plan[a] = plan_string(m->plan[a]);
        tune_store(key, best_v, best_fc, best_t1, chosen);
        return DSX_OK;
    });
}

dsx_status dsx_tune_set(dsx_model m, const int32_t choice[3])
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!choice) return fail(DSX_ERR_ARG, "null choice");
        const int v = choice[0], fc = choice[1], t1 = choice[2];
        if (!(v == 0 || v == 2 || v == 3 || v == 4 || v == 5) || (v != 0 && m->kind != DSX_NUCLEAR))
            return fail(DSX_ERR_ARG, "recombination form must be 0, or 2, 3, 4, 5 on a nuclear model");
        if (v == 5 && !direct_form_applies(m))
            return fail(DSX_ERR_ARG, "the direct form (5) needs Taylor order 0 and no |Q|-dependent scattering factor");
        if (!(fc == 0 || fc == 1 || fc == 2 || fc == 4))
            return fail(DSX_ERR_ARG, "FFT fields per plane block must be 0, 1, 2 or 4");
        if (t1 < 1 || t1 > 64) return fail(DSX_ERR_ARG, "filter planes per block must be in 1..64");
        m->tune_recomb_variant = v; m->tune_fchunk = fc; m->tune_lanczos_t1 = t1;
        m->tuned = true;
        return DSX_OK;
    });
}

dsx_status dsx_tune_query(dsx_model m, int32_t choice[3], int32_t* tuned)
{
    if (!m) return fail(DSX_ERR_ARG, "null model");
    if (!choice || !tuned) return fail(DSX_ERR_ARG, "null output");
    choice[0] = m->tune_recomb_variant;
    choice[1] = m->tune_fchunk;
    choice[2] = m->tune_lanczos_t1;
    *tuned = m->tuned ? 1 : 0;
    return DSX_OK;
}

dsx_status dsx_tune_set_fft(dsx_model m, const int32_t* radices, int32_t col_tile)
{
    return guarded([&]() -> dsx_status {
        dsx_status s = check_direct(m);
        if (s != DSX_OK) return s;
        if (!(col_tile == 0 || col_tile == 16 || col_tile == 32 || col_tile == 64))
            return fail(DSX_ERR_ARG, "the axis-1 column tile must be 0, 16, 32 or 64");
        if (col_tile && sizeof(float2) * (size_t)m->n[0] * (1 + 2 * (size_t)col_tile) > 160 * 1024)
            return fail(DSX_ERR_ARG, "the axis-1 column tile does not fit the LDS at this edge");
        AxisPlan np[3] = {m->plan[0], m->plan[1], m->plan[2]};
        if (radices) {
            for (int a = 0; a < 3; ++a) {
                AxisPlan p{};
                p.n = m->n[a];
                for (int i = 0; i < kMaxRadices && radices[a * kMaxRadices + i] != 0; ++i)
                    p.rad[p.nrad++] = radices[a * kMaxRadices + i];
                if (m->n[a] == 1 && p.nrad == 0) { np[a] = p; continue; }
                if (!plan_valid(p))
                    return fail(DSX_ERR_ARG, "axis " + std::to_string(a + 1) +
                                             ": radices must be 2, 4 or odd, with product n");
                np[a] = p;
            }
        }
        for (int a = 0; a < 3; ++a) m->plan[a] = np[a];
        m->tune_tc = col_tile;
        m->dirty = true;      // spectra are recomputed with the new plans
        m->tuned = true;
        return DSX_OK;
    });
}

dsx_status dsx_tune_query_fft(dsx_model m, int32_t* radices, int32_t* col_tile)
{
    if (!m) return fail(DSX_ERR_ARG, "null model");
    if (!radices || !col_tile) return fail(DSX_ERR_ARG, "null output");
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < kMaxRadices; ++i)
            radices[a * kMaxRadices + i] = i < m->plan[a].nrad ? m->plan[a].rad[i] : 0;
    *col_tile = m->tune_tc;
    return DSX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------- batches
namespace {

// One kernel node of a batch graph: a model's launch, or the launches of several
// models merged over a descriptor table.
struct BatchNode {
    const void* fn = nullptr;
    unsigned grid = 0, block = 0, lds = 0;
    bool merged = false;
    std::vector<unsigned char> params;     // single launch: its parameter block
    std::vector<int> members;              // merged: the models, in descriptor order
    std::vector<unsigned> counts;          // merged: each model's own grid
    std::vector<int> recs;                 // merged: each model's record index
    size_t tab_off = 0, slot_off = 0;      // merged: its arrays in the graph's device block
    std::vector<int> deps;                 // nodes holding the members' previous launches
};

struct BatchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* dmem = nullptr;                  // descriptor tables and slot maps
    int dispatches = 0, merged_nodes = 0, spill_kept = 0;
};

void free_graph(BatchGraph& g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    if (g.dmem) (void)hipFree(g.dmem);
    g = BatchGraph{};
}

// Position of a step in the path: launches of one step are merged, a step's nodes of
// different kernels run side by side.
int stage_rank(const char* s)
{
    static const char* const order[] = {"sums", "dw_sums", "dw_mean", "fft_planes", "fft_axis2",
                                        "fft_axis1", "recombine", "bragg", "lanczos"};
    for (int i = 0; i < (int)(sizeof(order) / sizeof(order[0])); ++i)
        if (std::strcmp(s, order[i]) == 0) return i;
    return (int)(sizeof(order) / sizeof(order[0]));
}

// A merged kernel is used only where it keeps the single kernel's registers in
// registers: no more private (spill) memory per lane than the single form.
bool merge_keeps_registers(const void* one, const void* merged)
{
    hipFuncAttributes a{}, b{};
    if (hipFuncGetAttributes(&a, one) != hipSuccess || hipFuncGetAttributes(&b, merged) != hipSuccess) return false;
    return b.localSizeBytes <= a.localSizeBytes;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Plan the kernel nodes of recorded sequences: merged (launches of a step that share a
// kernel, block size and LDS class become one node) or one node per launch.  Nodes come
// out in an order that respects every dependency, so issuing them in order on one stream
// is also valid.
dsx_status plan_nodes(const std::vector<std::vector<LaunchRec>>& seq, bool merge, std::vector<BatchNode>& nodes,
                      int* spill_kept_out)
{
    const int n = (int)seq.size();
    std::vector<size_t> head(n, 0);
    std::vector<int> last(n, -1);
    nodes.clear();
    int spill_kept = 0;
    for (;;) {
        int best = INT_MAX;
        for (int i = 0; i < n; ++i)
            if (head[i] < seq[i].size()) best = std::min(best, stage_rank(seq[i][head[i]].stage));
        if (best == INT_MAX) break;
        // the heads of this step, grouped by kernel, block size and the number of blocks
        // the LDS admits per CU (a node takes its members' largest LDS: members of one
        // class keep their occupancy), in model order
        std::vector<std::pair<std::tuple<const void*, unsigned, unsigned>, std::vector<int>>> groups;
        for (int i = 0; i < n; ++i) {
            if (head[i] >= seq[i].size()) continue;
            const LaunchRec& r = seq[i][head[i]];
            if (stage_rank(r.stage) != best) continue;
            const unsigned per_cu = r.lds ? std::min(64u, (160u * 1024u) / r.lds) : 64u;
            const auto key = std::make_tuple(r.merged, r.block, per_cu);
            auto g = std::find_if(groups.begin(), groups.end(), [&](const auto& x) { return x.first == key; });
            if (g == groups.end()) groups.push_back({key, {i}});
            else g->second.push_back(i);
        }
        for (auto& g : groups) {
            const std::vector<int>& mem = g.second;
            const LaunchRec& r0 = seq[mem[0]][head[mem[0]]];
            bool m = merge && mem.size() > 1;
            if (m && !merge_keeps_registers(r0.one, r0.merged)) {
                m = false;
                spill_kept += (int)mem.size();
            }
            if (!m) {
                for (int i : mem) {
                    const LaunchRec& r = seq[i][head[i]];
                    BatchNode nd;
                    nd.fn = r.one; nd.grid = r.grid; nd.block = r.block; nd.lds = r.lds;
                    nd.params = r.params;
                    if (last[i] >= 0) nd.deps.push_back(last[i]);
                    last[i] = (int)nodes.size();
                    ++head[i];
                    nodes.push_back(std::move(nd));
                }
                continue;
            }
            BatchNode nd;
            nd.fn = r0.merged; nd.block = r0.block; nd.merged = true;
            for (int i : mem) {
                const LaunchRec& r = seq[i][head[i]];
                if (r.params.size() != r0.params.size()) return fail(DSX_ERR_STATE, "batch: mismatched parameter blocks");
                nd.members.push_back(i);
                nd.counts.push_back(r.grid);
                nd.recs.push_back((int)head[i]);
                // every model's range starts at a multiple of 8 blocks: blocks keep their XCD
                const unsigned long long g8 = (unsigned long long)nd.grid + ((r.grid + 7u) & ~7u);
                if (g8 > 0x7fffffffULL) return fail(DSX_ERR_UNSUPPORTED, "batch: merged grid too large");
                nd.grid = (unsigned)g8;
                nd.lds = std::max(nd.lds, r.lds);
                if (last[i] >= 0 && std::find(nd.deps.begin(), nd.deps.end(), last[i]) == nd.deps.end())
                    nd.deps.push_back(last[i]);
            }
            for (int i : mem) { last[i] = (int)nodes.size(); ++head[i]; }
            nodes.push_back(std::move(nd));
        }
    }
    *spill_kept_out = spill_kept;
    return DSX_OK;
}

// Device bytes of the merged nodes' descriptor arrays and slot maps (sets their offsets).
size_t layout_nodes(const std::vector<std::vector<LaunchRec>>& seq, std::vector<BatchNode>& nodes)
{
    size_t bytes = 0;
    for (BatchNode& nd : nodes) {
        if (!nd.merged) continue;
        nd.tab_off = bytes;
        bytes = align256(bytes + nd.members.size() * seq[nd.members[0]][nd.recs[0]].params.size());
        nd.slot_off = bytes;
        bytes = align256(bytes + (size_t)(nd.grid / 8) * sizeof(Slot));
    }
    return bytes;
}

// Write the descriptor arrays and slot maps of the merged nodes into host memory of the
// size layout_nodes gave.
void fill_nodes(const std::vector<std::vector<LaunchRec>>& seq, const std::vector<BatchNode>& nodes, unsigned char* host,
                size_t bytes)
{
    std::memset(host, 0, bytes);
    for (const BatchNode& nd : nodes) {
        if (!nd.merged) continue;
        const size_t ps = seq[nd.members[0]][nd.recs[0]].params.size();
        Slot* sl = reinterpret_cast<Slot*>(host + nd.slot_off);
        int first = 0;
        for (size_t d = 0; d < nd.members.size(); ++d) {
            const LaunchRec& r = seq[nd.members[d]][nd.recs[d]];
            std::memcpy(host + nd.tab_off + d * ps, r.params.data(), ps);
            const int span = (int)((nd.counts[d] + 7u) & ~7u);
            for (int b = first; b < first + span; b += 8)
                sl[b / 8] = Slot{(int32_t)d, first, (int32_t)nd.counts[d], 0};
            first += span;
        }
    }
}

// Build the graph of the recorded sequences.
dsx_status build_batch_graph(const std::vector<std::vector<LaunchRec>>& seq, bool merge, BatchGraph& out)
{
    std::vector<BatchNode> nodes;
    int spill_kept = 0;
    dsx_status ps = plan_nodes(seq, merge, nodes, &spill_kept);
    if (ps != DSX_OK) return ps;
    const size_t bytes = layout_nodes(seq, nodes);
    BatchGraph g;
    auto bail = [&](dsx_status st) { free_graph(g); return st; };
    hipError_t e = hipSuccess;
    if (bytes) {
        std::vector<unsigned char> host(bytes, 0);
        fill_nodes(seq, nodes, host.data(), bytes);
        if ((e = hipMalloc(&g.dmem, bytes)) != hipSuccess) return bail(fail(DSX_ERR_NOMEM, hipGetErrorString(e)));
        if ((e = hipMemcpy(g.dmem, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
    }
    if ((e = hipGraphCreate(&g.graph, 0)) != hipSuccess) return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
    std::vector<hipGraphNode_t> gn(nodes.size(), nullptr);
    std::vector<hipGraphNode_t> deps;
    for (size_t k = 0; k < nodes.size(); ++k) {
        BatchNode& nd = nodes[k];
        if (nd.lds > 65536 &&
            (e = hipFuncSetAttribute(nd.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)nd.lds)) != hipSuccess)
            return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
        void* tab = g.dmem ? (char*)g.dmem + nd.tab_off : nullptr;
        void* slots = g.dmem ? (char*)g.dmem + nd.slot_off : nullptr;
        void* margs[2] = {&tab, &slots};
        void* sargs[1] = {nd.params.data()};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(nd.fn);
        kp.gridDim = dim3(nd.grid);
        kp.blockDim = dim3(nd.block);
        kp.sharedMemBytes = nd.lds;
        kp.kernelParams = nd.merged ? margs : sargs;
        kp.extra = nullptr;
        deps.clear();
        for (int d : nd.deps) deps.push_back(gn[d]);
        if ((e = hipGraphAddKernelNode(&gn[k], g.graph, deps.empty() ? nullptr : deps.data(), deps.size(), &kp)) != hipSuccess)
            return bail(fail(DSX_ERR_DEVICE, std::string("graph node: ") + hipGetErrorString(e)));
        ++g.dispatches;
        if (nd.merged) ++g.merged_nodes;
    }
    if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess)
        return bail(fail(DSX_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e)));
    g.spill_kept = spill_kept;
    out = g;
    return DSX_OK;
}

}  // namespace

struct dsx_batch_s {
    std::vector<dsx_model> models;
    std::vector<float*> outs;
    int lanczos_m = 0, oversample = 1;
    int mode = DSX_BATCH_PER_MODEL, launches = 0, merged_form_dispatches = -1;
    float per_model_ms = -1.f, merged_ms = -1.f;
    hipStream_t cap = nullptr;
    BatchGraph g;
};

namespace {

void free_batch(dsx_batch b)
{
    free_graph(b->g);
    if (b->cap) (void)hipStreamDestroy(b->cap);
}

// Each model's launch sequence, recorded (nothing runs).  The models' dirty flags are
// kept: recording computes nothing.
dsx_status record_batch(dsx_batch b, std::vector<std::vector<LaunchRec>>& seq)
{
    const int n = (int)b->models.size();
    seq.assign(n, {});
    for (int i = 0; i < n; ++i) {
        dsx_model m = b->models[i];
        const bool dirty = m->dirty;
        Recorder r;
        struct Reset { ~Reset() { g_recorder = nullptr; } } reset;
        g_recorder = &r;
        const dsx_status s = b->lanczos_m ? enqueue_filter(m, b->lanczos_m, b->oversample, b->outs[i], b->cap, true)
                                          : enqueue_intensity(m, b->outs[i], b->cap, true);
        g_recorder = nullptr;
        m->dirty = dirty;
        if (s != DSX_OK) return s;
        seq[i] = std::move(r.recs);
    }
    return DSX_OK;
}

// Best of three replays of graph g on stream st (after one untimed replay), ms.
float time_graph(const BatchGraph& g, hipStream_t st)
{
    if (hipGraphLaunch(g.exec, st) != hipSuccess) return -1.f;
    return time_min(st, 3, [&]() -> dsx_status {
        return hipGraphLaunch(g.exec, st) == hipSuccess ? DSX_OK : DSX_ERR_DEVICE;
    });
}

}  // namespace

extern "C" {

dsx_status dsx_batch_create_mode(const dsx_model* models, int32_t n, int32_t lanczos_m, int32_t oversample,
                                 float* const* outs, int32_t mode, dsx_batch* out)
{
    return guarded([&]() -> dsx_status {
        if (!models || !outs || !out || n < 1) return fail(DSX_ERR_ARG, "models, outs and out are required, n >= 1");
        if (mode != DSX_BATCH_AUTO && mode != DSX_BATCH_PER_MODEL && mode != DSX_BATCH_MERGED)
            return fail(DSX_ERR_ARG, "unknown batch mode");
        *out = nullptr;
        dsx_status s;
        if (lanczos_m != 0 && (s = check_filter_args(lanczos_m, oversample)) != DSX_OK) return s;
        for (int i = 0; i < n; ++i) {
            if ((s = check_direct(models[i])) != DSX_OK) return s;
            if ((s = ready(models[i])) != DSX_OK) return s;
            if (!outs[i]) return fail(DSX_ERR_ARG, "outs[" + std::to_string(i) + "] is NULL");
            for (int j = 0; j < i; ++j)
                if (models[j] == models[i]) return fail(DSX_ERR_ARG, "a model appears twice in the batch");
        }
        dsx_batch b = new (std::nothrow) dsx_batch_s();
        if (!b) return fail(DSX_ERR_NOMEM, "host allocation failed");
        auto bail = [&](dsx_status st) { free_batch(b); delete b; return st; };
        try {
            b->models.assign(models, models + n);
            b->outs.assign(outs, outs + n);
        } catch (...) {
            delete b;
            throw;
        }
        b->lanczos_m = lanczos_m;
        b->oversample = lanczos_m ? oversample : 1;
        hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
        // plan and tune (allocations and uploads happen here, never in the graph)
        for (int i = 0; i < n; ++i) {
            dsx_model m = b->models[i];
            if (!m->tuned && (s = dsx_autotune(m, lanczos_m, b->cap)) != DSX_OK) return bail(s);
            if ((s = prepare_intensity(m)) != DSX_OK) return bail(s);
            if (lanczos_m && (s = prepare_filter(m, lanczos_m, b->oversample)) != DSX_OK) return bail(s);
        }
        if ((e = hipStreamSynchronize(b->cap)) != hipSuccess) return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
        std::vector<std::vector<LaunchRec>> seq;
        if ((s = record_batch(b, seq)) != DSX_OK) return bail(s);
        for (const auto& q : seq) b->launches += (int)q.size();
        if ((s = build_batch_graph(seq, mode != DSX_BATCH_PER_MODEL, b->g)) != DSX_OK) return bail(s);
        // a graph without merged nodes is the per-model form
        b->mode = b->g.merged_nodes > 0 ? DSX_BATCH_MERGED : DSX_BATCH_PER_MODEL;
        if (mode != DSX_BATCH_PER_MODEL) b->merged_form_dispatches = b->g.dispatches;
        if (mode == DSX_BATCH_AUTO && b->mode == DSX_BATCH_MERGED) {
            // time both forms on the device and keep the faster
            BatchGraph pm;
            if ((s = build_batch_graph(seq, false, pm)) != DSX_OK) return bail(s);
            for (dsx_model m : b->models) (void)hipStreamSynchronize(m->last_stream);
            b->merged_ms = time_graph(b->g, b->cap);
            b->per_model_ms = time_graph(pm, b->cap);
            if ((e = hipStreamSynchronize(b->cap)) != hipSuccess || b->merged_ms < 0.f || b->per_model_ms < 0.f) {
                free_graph(pm);
                return bail(fail(DSX_ERR_DEVICE, "batch: timing the graphs failed"));
            }
            if (b->per_model_ms < b->merged_ms) {
                std::swap(b->g, pm);
                b->mode = DSX_BATCH_PER_MODEL;
            }
            free_graph(pm);
        }
        for (dsx_model m : b->models) ++m->pins;
        *out = b;
        return DSX_OK;
    });
}

dsx_status dsx_batch_create(const dsx_model* models, int32_t n, int32_t lanczos_m, int32_t oversample,
                            float* const* outs, dsx_batch* out)
{
    return dsx_batch_create_mode(models, n, lanczos_m, oversample, outs, DSX_BATCH_AUTO, out);
}

dsx_status dsx_batch_query(dsx_batch b, dsx_batch_info* info)
{
    return guarded([&]() -> dsx_status {
        if (!b || !info) return fail(DSX_ERR_ARG, "batch and info are required");
        info->mode = b->mode;
        info->launches = b->launches;
        info->dispatches = b->g.dispatches;
        info->merged_nodes = b->g.merged_nodes;
        info->unmerged_spill = b->g.spill_kept;
        info->merged_form_dispatches = b->merged_form_dispatches;
        info->per_model_ms = b->per_model_ms;
        info->merged_ms = b->merged_ms;
        return DSX_OK;
    });
}

dsx_status dsx_batch_run(dsx_batch b, void* hip_stream)
{
    return guarded([&]() -> dsx_status {
        if (!b) return fail(DSX_ERR_ARG, "batch is NULL");
        for (dsx_model m : b->models) {
            dsx_status s = check_model(m);
            if (s != DSX_OK) return s;
        }
        hipStream_t st = (hipStream_t)hip_stream;
        for (dsx_model m : b->models) {
            dsx_status s = follow(m, st);
            if (s != DSX_OK) return s;
        }
        const hipError_t e = hipGraphLaunch(b->g.exec, st);
        if (e != hipSuccess) {
            for (dsx_model m : b->models) m->failed = true;
            return fail(DSX_ERR_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        }
        for (dsx_model m : b->models) m->dirty = false;
        return DSX_OK;
    });
}

dsx_status dsx_batch_destroy(dsx_batch b)
{
    return guarded([&]() -> dsx_status {
        if (!b) return fail(DSX_ERR_ARG, "batch is NULL");
        for (dsx_model m : b->models) { (void)hipStreamSynchronize(m->last_stream); --m->pins; }
        free_batch(b);
        delete b;
        return DSX_OK;
    });
}

dsx_status dsx_destroy_model(dsx_model m)
{
    return guarded([&]() -> dsx_status {
        if (!m) return fail(DSX_ERR_ARG, "model is NULL");
        if (m->server) return fail(DSX_ERR_ARG, "the model belongs to a server: dsx_server_destroy releases it");
        if (m->pins) return fail(DSX_ERR_BUSY, "the model is recorded in a batch; destroy the batch first");
        (void)hipStreamSynchronize(m->last_stream);
        free_model(m);
        delete m;
        return DSX_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------- serving
namespace {

using Clock = std::chrono::steady_clock;

// First-fit sub-allocator over the server's device arena, in 256-byte granules.


struct Request {
    int64_t ticket = 0;
    dsx_request r{};
    size_t ws = 0, off = 0;     // workspace bytes and its arena offset
    size_t x_bytes = 0;         // spectra part of the workspace
    int64_t voxels = 0;
    Clock::time_point t_submit;
    int bypassed = 0;           // later requests admitted before this one
};

struct Finished {
    dsx_status status;
    std::string msg;
};

constexpr int kMaxBypass = 64;
// Requests up to this many output voxels may share a merged round (their launches are
// short, so a round saves launch and tail time); larger ones run alone on their slot,
// beside the other slots' work.
constexpr int64_t kRoundMaxVoxels = 1 << 20;

}  // namespace

struct dsx_server_s {
    int device = 0;
    int nslots = 0, capacity = 0;
    char* arena_mem = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<char> busy;
    std::vector<std::vector<Request>> running;   // per slot: the requests of its round
    int max_round = 16;
    // per slot: pinned host and device staging of a round's descriptor tables
    std::vector<unsigned char*> hstage;
    std::vector<void*> dstage;
    size_t stage_bytes = 0;
    std::deque<Request> queue;
    std::vector<dsx_model> models;
    std::set<dsx_model> active;        // models with a request on the device
    std::map<int64_t, Finished> finished;
    std::set<int64_t> pending;         // queued or running tickets
    int64_t next_ticket = 1;
    bool stop = false;
    std::mutex mu;
    std::condition_variable wake;      // the dispatcher: new request or stop
    std::condition_variable done;      // waiters: a request finished
    std::thread worker;
    // statistics since the last reset
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, voxels = 0;
    std::vector<double> lat_ms;
    bool have_first = false;
    Clock::time_point first_submit, last_done;
    int in_flight = 0, peak_in_flight = 0;
    int64_t rounds = 0, round_requests = 0;
};

namespace {


// Workspace of one request: spectra, partial lattice sums and, filtered, the grown box.
size_t request_workspace(dsx_model m, int lm, size_t* x_bytes)
{
    *x_bytes = Arena::round(m->spectrum_bytes);
    size_t ws = *x_bytes + Arena::round(m->partial_bytes);
    if (lm >= 2) ws += Arena::round(ext_elems(filter_box(m->box, lm)) * sizeof(float));
    return ws;
}

// Enqueues an admitted request on stream st (its site copy, then its kernels; with a
// recorder set the kernels are recorded instead) (dispatcher thread).
dsx_status enqueue_request(dsx_server s, const Request& q, hipStream_t st)
{
    dsx_model m = q.r.model;
    dsx_status rs = check_model(m);
    if (rs != DSX_OK) return rs;
    const int lm = q.r.lanczos_m, sv = lm >= 2 ? q.r.oversample : 1;
    char* base = s->arena_mem + q.off;
    m->d_X = reinterpret_cast<float2*>(base);
    m->d_partial = reinterpret_cast<double*>(base + q.x_bytes);
    if (lm >= 2) {
        m->d_ext = reinterpret_cast<float*>(base + q.x_bytes + Arena::round(m->partial_bytes));
        m->ext_cap = ext_elems(filter_box(m->box, lm));
    }
    rs = follow(m, st);
    if (rs == DSX_OK && q.r.config >= 0) {
        const hipMemcpyKind kind = q.r.where == DSX_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        const size_t per = (size_t)m->S * m->ncell;
        const float* vec = m->kind == DSX_MAGNETIC ? q.r.spin : q.r.disp;
        hipError_t e = hipSuccess;
        if (m->has_occ) e = hipMemcpyAsync(m->d_occ + per * q.r.config, q.r.occ, per * sizeof(float), kind, st);
        if (e == hipSuccess && vec)
            e = hipMemcpyAsync(m->d_vec + 3 * per * q.r.config, vec, 3 * per * sizeof(float), kind, st);
        if (e == hipSuccess && m->dw_order > 0)
            e = hipMemcpyAsync(m->d_dsp + 3 * per * q.r.config, q.r.disp, 3 * per * sizeof(float), kind, st);
        if (e != hipSuccess) { m->failed = true; rs = fail(DSX_ERR_DEVICE, std::string("site upload: ") + hipGetErrorString(e)); }
        else m->set[q.r.config] = 1;
    }
    if (rs == DSX_OK) rs = ready(m);
    if (rs == DSX_OK) rs = lm >= 2 ? prepare_filter(m, lm, sv) : prepare_intensity(m);
    if (rs == DSX_OK)
        rs = lm >= 2 ? enqueue_filter(m, lm, sv, q.r.out, st, true) : enqueue_intensity(m, q.r.out, st, true);
    // the arena range belongs to the request, not the model
    m->d_X = nullptr; m->d_partial = nullptr; m->d_ext = nullptr; m->ext_cap = 0;
    m->dirty = true;
    return rs;
}

// Enqueues an admitted request on stream st and records ev after it (dispatcher thread).
dsx_status launch_request(dsx_server s, const Request& q, hipStream_t st, hipEvent_t ev)
{
    dsx_status rs = enqueue_request(s, q, st);
    if (rs == DSX_OK) {
        const hipError_t e = hipEventRecord(ev, st);
        if (e != hipSuccess) { q.r.model->failed = true; rs = fail(DSX_ERR_DEVICE, hipGetErrorString(e)); }
    }
    if (rs != DSX_OK) (void)hipStreamSynchronize(st);   // nothing may still use the range
    return rs;
}

// A round of several requests on one slot: every request's site copy is enqueued and its
// kernels recorded, then the kernels of all of them run as merged launches on the slot's
// stream, the descriptor tables copied from the slot's pinned staging.  status[i] is the
// outcome of request i; the event is recorded after the round.  Returns DSX_OK when the
// round was enqueued (some requests may have failed before any kernel of theirs).
dsx_status launch_round(dsx_server s, int slot, std::vector<dsx_status>& status, std::vector<std::string>& msg)
{
    std::vector<Request>& reqs = s->running[slot];
    const hipStream_t st = s->streams[slot];
    const int n = (int)reqs.size();
    status.assign(n, DSX_OK);
    msg.assign(n, std::string());
    std::vector<std::vector<LaunchRec>> seq;
    std::vector<int> who;                       // request of each recorded sequence
    for (int i = 0; i < n; ++i) {
        Recorder r;
        struct Reset { ~Reset() { g_recorder = nullptr; } } reset;
        g_recorder = &r;
        const dsx_status rs = enqueue_request(s, reqs[i], st);
        g_recorder = nullptr;
        if (rs != DSX_OK) { status[i] = rs; msg[i] = dsx_last_error(); continue; }
        seq.push_back(std::move(r.recs));
        who.push_back(i);
    }
    hipError_t e = hipSuccess;
    dsx_status rs = DSX_OK;
    if (!seq.empty()) {
        std::vector<BatchNode> nodes;
        int kept = 0;
        rs = plan_nodes(seq, true, nodes, &kept);
        size_t bytes = rs == DSX_OK ? layout_nodes(seq, nodes) : 0;
        if (rs == DSX_OK && bytes > s->stage_bytes) {   // tables too large: the round runs unmerged
            rs = plan_nodes(seq, false, nodes, &kept);
            bytes = 0;
        }
        if (rs == DSX_OK && bytes) {
            fill_nodes(seq, nodes, s->hstage[slot], bytes);
            e = hipMemcpyAsync(s->dstage[slot], s->hstage[slot], bytes, hipMemcpyHostToDevice, st);
        }
        for (size_t k = 0; rs == DSX_OK && e == hipSuccess && k < nodes.size(); ++k) {
            BatchNode& nd = nodes[k];
            if (nd.lds > 65536 &&
                (e = hipFuncSetAttribute(nd.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)nd.lds)) != hipSuccess)
                break;
            void* tab = (char*)s->dstage[slot] + nd.tab_off;
            void* slots = (char*)s->dstage[slot] + nd.slot_off;
            void* margs[2] = {&tab, &slots};
            void* sargs[1] = {nd.params.data()};
            e = hipLaunchKernel(nd.fn, dim3(nd.grid), dim3(nd.block), nd.merged ? margs : sargs, nd.lds, st);
        }
    }
    if (e == hipSuccess && rs == DSX_OK) e = hipEventRecord(s->events[slot], st);
    if (e != hipSuccess || rs != DSX_OK) {
        const std::string m = e != hipSuccess ? std::string(hipGetErrorString(e)) : std::string(dsx_last_error());
        for (int i : who) {
            reqs[i].r.model->failed = e != hipSuccess;
            status[i] = e != hipSuccess ? DSX_ERR_DEVICE : rs;
            msg[i] = m;
        }
        (void)hipStreamSynchronize(st);   // nothing may still use the arena ranges
        return status.empty() ? DSX_OK : status[0];
    }
    return DSX_OK;
}

// Bookkeeping of a request that left the device (lock held).
void finish_request(dsx_server s, const Request& q, dsx_status st, const std::string& msg)
{
    s->arena.release(q.off, q.ws);
    s->active.erase(q.r.model);
    --q.r.model->queued;
    s->pending.erase(q.ticket);
    s->finished[q.ticket] = Finished{st, msg};
    if (st == DSX_OK) {
        const Clock::time_point now = Clock::now();
        ++s->completed;
        s->voxels += q.voxels;
        s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - q.t_submit).count());
        s->last_done = now;
    } else {
        ++s->failed;
    }
}

void serve(dsx_server s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool changed = false;
        for (int i = 0; i < s->nslots; ++i) {
            if (!s->busy[i]) continue;
            const hipError_t e = hipEventQuery(s->events[i]);
            if (e == hipErrorNotReady) continue;
            dsx_status st = DSX_OK;
            std::string msg;
            if (e != hipSuccess) {
                st = DSX_ERR_DEVICE;
                msg = hipGetErrorString(e);
            }
            for (Request& q : s->running[i]) {
                if (e != hipSuccess) q.r.model->failed = true;
                finish_request(s, q, st, msg);
                --s->in_flight;
            }
            s->running[i].clear();
            s->busy[i] = 0;
            changed = true;
        }
        // admission: first come first served among requests whose workspace fits and
        // whose model is idle; a request that fits may pass one that does not yet.  A
        // free slot takes a round of up to max_round such requests.
        for (;;) {
            int slot = -1;
            for (int i = 0; i < s->nslots && slot < 0; ++i)
                if (!s->busy[i]) slot = i;
            if (slot < 0 || s->queue.empty()) break;
            std::set<dsx_model> waiting;   // models with an earlier request still queued
            std::vector<Request>& round = s->running[slot];
            round.clear();
            bool closed = false;           // a large request runs alone
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)round.size() < s->max_round && !closed;) {
                if (it != s->queue.begin() && s->queue.front().bypassed >= kMaxBypass) break;
                dsx_model m = it->r.model;
                const bool large = it->voxels > kRoundMaxVoxels;
                if (large && !round.empty()) {   // (its model's later requests wait behind it)
                    waiting.insert(m);
                    ++it;
                    continue;
                }
                size_t off = 0;
                if (s->active.count(m) || waiting.count(m) || !s->arena.alloc(it->ws, &off)) {
                    waiting.insert(m);
                    ++it;
                    continue;
                }
                it->off = off;
                for (auto jt = s->queue.begin(); jt != it; ++jt) ++jt->bypassed;
                s->active.insert(m);
                round.push_back(std::move(*it));
                it = s->queue.erase(it);
                closed = large;
            }
            if (round.empty()) break;
            s->busy[slot] = 1;
            s->in_flight += (int)round.size();
            s->peak_in_flight = std::max(s->peak_in_flight, s->in_flight);
            ++s->rounds;
            s->round_requests += (int64_t)round.size();
            lk.unlock();
            std::vector<dsx_status> sts;
            std::vector<std::string> msgs;
            if (round.size() == 1) {
                sts.assign(1, launch_request(s, round[0], s->streams[slot], s->events[slot]));
                msgs.assign(1, sts[0] == DSX_OK ? std::string() : std::string(dsx_last_error()));
            } else {
                (void)launch_round(s, slot, sts, msgs);
            }
            lk.lock();
            // requests that failed before any of their kernels left the round now
            std::vector<Request> keep;
            for (size_t i = 0; i < round.size(); ++i) {
                if (sts[i] == DSX_OK) { keep.push_back(std::move(round[i])); continue; }
                finish_request(s, round[i], sts[i], msgs[i]);
                --s->in_flight;
            }
            round.swap(keep);
            if (round.empty()) s->busy[slot] = 0;
            changed = true;
        }
        if (changed) s->done.notify_all();
        if (s->stop && s->queue.empty() && s->in_flight == 0) break;
        if (s->in_flight == 0)
            s->wake.wait(lk, [&] { return s->stop || !s->queue.empty(); });
        else
            s->wake.wait_for(lk, std::chrono::microseconds(50));
    }
    s->done.notify_all();
}

void free_server(dsx_server s)
{
    for (dsx_model m : s->models) { free_model(m); delete m; }
    for (auto e : s->events) if (e) (void)hipEventDestroy(e);
    for (auto st : s->streams) if (st) (void)hipStreamDestroy(st);
    for (auto h : s->hstage) if (h) (void)hipHostFree(h);
    for (auto d : s->dstage) if (d) (void)hipFree(d);
    dfree(s->arena_mem);
}

}  // namespace

extern "C" {

dsx_status dsx_server_create(const dsx_server_config* c, dsx_server* out)
{
    return guarded([&]() -> dsx_status {
        if (!c || !out) return fail(DSX_ERR_ARG, "config and out are required");
        *out = nullptr;
        if (c->slots < 1 || c->slots > 16) return fail(DSX_ERR_ARG, "slots must be in 1..16");
        if (c->queue_capacity < 1) return fail(DSX_ERR_ARG, "queue_capacity must be >= 1");
        if (c->arena_bytes < 1) return fail(DSX_ERR_ARG, "arena_bytes must be >= 1");
        if (c->max_round < 0 || c->max_round > 64) return fail(DSX_ERR_ARG, "max_round must be in 0..64");
        dsx_server s = new (std::nothrow) dsx_server_s();
        if (!s) return fail(DSX_ERR_NOMEM, "host allocation failed");
        auto bail = [&](dsx_status st) { free_server(s); delete s; return st; };
        (void)hipGetDevice(&s->device);
        s->nslots = c->slots;
        s->capacity = c->queue_capacity;
        const size_t bytes = Arena::round((size_t)c->arena_bytes);
        hipError_t e = hipMalloc(&s->arena_mem, bytes);
        if (e == hipErrorOutOfMemory) { (void)hipGetLastError(); return bail(fail(DSX_ERR_NOMEM, "out of device memory for the arena")); }
        if (e != hipSuccess) return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
        s->arena.init(bytes);
        s->streams.assign(s->nslots, nullptr);
        s->events.assign(s->nslots, nullptr);
        s->busy.assign(s->nslots, 0);
        s->running.resize(s->nslots);
        s->max_round = c->max_round == 0 ? 16 : c->max_round;
        s->stage_bytes = s->max_round > 1 ? (size_t)4 << 20 : 0;
        s->hstage.assign(s->nslots, nullptr);
        s->dstage.assign(s->nslots, nullptr);
        for (int i = 0; i < s->nslots; ++i) {
            if ((e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming)) != hipSuccess)
                return bail(fail(DSX_ERR_DEVICE, hipGetErrorString(e)));
            if (s->stage_bytes &&
                ((e = hipHostMalloc((void**)&s->hstage[i], s->stage_bytes, hipHostMallocDefault)) != hipSuccess ||
                 (e = hipMalloc(&s->dstage[i], s->stage_bytes)) != hipSuccess))
                return bail(fail(DSX_ERR_NOMEM, std::string("round staging: ") + hipGetErrorString(e)));
        }
        try {
            s->worker = std::thread(serve, s);
        } catch (...) {
            return bail(fail(DSX_ERR_NOMEM, "cannot start the dispatcher thread"));
        }
        *out = s;
        return DSX_OK;
    });
}

dsx_status dsx_server_add_model(dsx_server s, const dsx_model_desc* d, dsx_model* out)
{
    return guarded([&]() -> dsx_status {
        if (!s) return fail(DSX_ERR_ARG, "server is NULL");
        dsx_status st = create_model_impl(d, true, out);
        if (st != DSX_OK) return st;
        (*out)->server = s;
        std::lock_guard<std::mutex> lk(s->mu);
        s->models.push_back(*out);
        return DSX_OK;
    });
}

dsx_status dsx_server_submit(dsx_server s, const dsx_request* r, int64_t* ticket)
{
    return guarded([&]() -> dsx_status {
        if (!s || !r || !ticket) return fail(DSX_ERR_ARG, "server, request and ticket are required");
        dsx_model m = r->model;
        dsx_status st = check_model(m);
        if (st != DSX_OK) return st;
        if (m->server != s) return fail(DSX_ERR_ARG, "the model does not belong to this server");
        if (!r->out) return fail(DSX_ERR_ARG, "out is NULL");
        if (r->lanczos_m != 0 && (st = check_filter_args(r->lanczos_m, r->oversample)) != DSX_OK) return st;
        if (!m->grid_set) return fail(DSX_ERR_STATE, "no output grid set");
        if (r->config >= m->M || r->config < -1) return fail(DSX_ERR_ARG, "config out of range");
        if (r->config >= 0) {
            if (r->where != DSX_HOST && r->where != DSX_DEVICE) return fail(DSX_ERR_ARG, "bad 'where'");
            if (m->has_occ && !r->occ) return fail(DSX_ERR_ARG, "occ is required (has_occ != 0)");
            const bool need_vec = m->kind == DSX_MAGNETIC || m->order > 0;
            if (need_vec && !(m->kind == DSX_MAGNETIC ? r->spin : r->disp))
                return fail(DSX_ERR_ARG, m->kind == DSX_MAGNETIC ? "spin is required" : "disp is required");
            if (m->dw_order > 0 && !r->disp) return fail(DSX_ERR_ARG, "disp is required (taylor_order > 0)");
        }
        Request q;
        q.r = *r;
        q.ws = request_workspace(m, r->lanczos_m, &q.x_bytes);
        if (q.ws > s->arena.size())
            return fail(DSX_ERR_NOMEM, "the request's workspace (" + std::to_string(q.ws) +
                                       " bytes) exceeds the server's arena");
        const int64_t sv = r->lanczos_m >= 2 ? r->oversample : 1;
        q.voxels = sv * m->box.cnt[0] * sv * m->box.cnt[1] * sv * (int64_t)m->box.cnt[2];
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(DSX_ERR_STATE, "the server is shutting down");
        if ((int)s->queue.size() >= s->capacity) {
            ++s->rejected;
            return fail(DSX_ERR_BUSY, "request queue full");
        }
        q.ticket = s->next_ticket++;
        q.t_submit = Clock::now();
        if (!s->have_first) { s->first_submit = q.t_submit; s->have_first = true; }
        ++m->queued;
        ++s->submitted;
        s->pending.insert(q.ticket);
        *ticket = q.ticket;
        s->queue.push_back(std::move(q));
        s->wake.notify_one();
        return DSX_OK;
    });
}

dsx_status dsx_server_wait(dsx_server s, int64_t ticket, int32_t timeout_ms, dsx_status* result)
{
    return guarded([&]() -> dsx_status {
        if (!s || !result) return fail(DSX_ERR_ARG, "server and result are required");
        std::unique_lock<std::mutex> lk(s->mu);
        auto ready_ = [&] { return s->finished.count(ticket) > 0 || !s->pending.count(ticket); };
        if (timeout_ms < 0) s->done.wait(lk, ready_);
        else s->done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready_);
        auto it = s->finished.find(ticket);
        if (it == s->finished.end()) {
            if (!s->pending.count(ticket)) return fail(DSX_ERR_ARG, "unknown or already retired ticket");
            return fail(DSX_ERR_BUSY, "the request has not finished");
        }
        *result = it->second.status;
        g_err = it->second.msg;
        s->finished.erase(it);
        return DSX_OK;
    });
}

dsx_status dsx_server_stats_read(dsx_server s, int32_t reset, dsx_server_stats* out)
{
    return guarded([&]() -> dsx_status {
        if (!s || !out) return fail(DSX_ERR_ARG, "server and out are required");
        std::lock_guard<std::mutex> lk(s->mu);
        dsx_server_stats z{};
        z.submitted = s->submitted; z.completed = s->completed; z.failed = s->failed; z.rejected = s->rejected;
        z.voxels = s->voxels;
        std::vector<double> l = s->lat_ms;
        if (!l.empty()) {
            std::sort(l.begin(), l.end());
            auto q = [&](double p) {   // nearest-rank percentile
                size_t k = (size_t)std::ceil(p * l.size());
                return l[std::min(l.size(), std::max<size_t>(k, 1)) - 1];
            };
            z.p50_ms = q(0.50);
            z.p99_ms = q(0.99);
            double t = 0;
            for (double v : l) t += v;
            z.mean_ms = t / l.size();
            z.max_ms = l.back();
            z.span_s = std::chrono::duration<double>(s->last_done - s->first_submit).count();
        }
        z.arena_bytes = (int64_t)s->arena.size();
        z.arena_peak_bytes = (int64_t)s->arena.peak();
        z.slots = s->nslots;
        z.peak_in_flight = s->peak_in_flight;
        z.rounds = s->rounds;
        z.round_requests = s->round_requests;
        *out = z;
        if (reset) {
            s->submitted = s->completed = s->failed = s->rejected = s->voxels = 0;
            s->rounds = s->round_requests = 0;
            s->lat_ms.clear();
            s->have_first = false;
            s->peak_in_flight = s->in_flight;
            s->arena.reset_peak();
        }
        return DSX_OK;
    });
}

dsx_status dsx_server_destroy(dsx_server s)
{
    return guarded([&]() -> dsx_status {
        if (!s) return fail(DSX_ERR_ARG, "server is NULL");
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->wake.notify_all();
        if (s->worker.joinable()) s->worker.join();
        for (auto st : s->streams) if (st) (void)hipStreamSynchronize(st);
        free_server(s);
        delete s;
        return DSX_OK;
    });
}

}  // extern "C"
