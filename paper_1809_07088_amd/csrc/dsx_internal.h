// Internal parameter blocks and launchers shared by the host runtime (api.cpp)
// and the gfx950 kernels (fft.hip, recombine.hip, lanczos.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace dsx {

constexpr int kMaxN = 256;        // supercell edge
constexpr int kMaxSites = 64;
constexpr int kMaxOrder = 16;
constexpr int kMaxMono = 969;     // monomials of total degree <= 16: C(19, 3)
// Taylor orders above this take the class form of the recombination with at most 8 H3
// per thread (the folded and parity forms and longer H3 runs are instantiated up to it)
constexpr int kMaxOrderFast = 8;
constexpr int kMaxRadices = 16;

// Mixed-radix factorisation of one FFT axis.
struct AxisPlan {
    int32_t n;
    int32_t nrad;
    int32_t rad[kMaxRadices];
};

// Number of monomials u1^p u2^q u3^r with p + q + r <= N.
__host__ __device__ constexpr int n_monomials(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
// Number of (q, r) pairs with q + r <= N.
__host__ __device__ constexpr int n_pairs(int N) { return (N + 1) * (N + 2) / 2; }
// Index of monomial (p, q, r), ordered by degree d, then p descending, then q descending.
__host__ __device__ constexpr int mono_index(int p, int q, int r) {
    return (p + q + r) * (p + q + r + 1) * (p + q + r + 2) / 6
         + (q + r) * (q + r + 1) / 2 + r;
}
// Index of the pair (q, r), ordered by e = q + r, then q descending.
__host__ __device__ constexpr int pair_index(int q, int r) { return (q + r) * (q + r + 1) / 2 + r; }

// ---------------------------------------------------------------------------- FP64 sums
// Lattice cells per block of the sums kernels (a multiple of 256, the block size):
// enough blocks to fill the chip, at most 8 cells per thread.
inline int sums_chunk(long long ncell, long long ms)
{
    long long per = (ncell * ms) / (256LL * 2048);
    per = per < 1 ? 1 : (per > 8 ? 8 : per);
    return (int)(256 * per);
}
struct SumsParams {
    const float* occ;     // [M][S][ncell] or null (delta = 1)
    const float* vec;     // [M][S][ncell][3] displacements (nuclear) or spins (magnetic)
    double* partial;      // [M*S][nchunk][T]
    double* sums;         // [M*S][T]
    int32_t M, S, ncell, T, kind, nchunk, chunk;
};

// ---------------------------------------------------------------------------- FFT
struct PlaneParams {
    const float* occ;     // [M][S][n1][n2][n3] or null
    const float* vec;     // [M][S][n1][n2][n3][3] or null
    const double* sums;   // [M*S][T] lattice sums (the field means are sums / ncell)
    float2* X;            // [M][n1][n2][S*F][nh]; this pass writes the R1 index in place of k1.
                          // Fields of a site are ordered by the pair (q, r) (e = q + r ascending,
                          // q descending), then p ascending, so that each p-run is contiguous.
    const float2* tw2;    // e^{+2 pi i t / n2}, t < n2
    const float2* tw3;    // e^{+2 pi i t / n3}, t < n3
    AxisPlan p2, p3;
    int32_t n1, n2, n3, nh, S, F, T, M, kind, first_mono;
    int32_t fchunk, nfchunk;
    int32_t npl;          // lattice planes per block (small planes; the rows kernel takes 1)
    int32_t buf_elems;    // complex elements per LDS ping-pong buffer
    int32_t row_pairs;    // > 0: the plane does not fit the LDS; blocks take this many row pairs
                          // and transform along axis 3 only (axis 2 follows in place)
    int32_t nrchunk;      // row-pair chunks per plane
    int8_t mono[3 * kMaxMono];   // exponents (p, q, r) of field f (spectra order)
};

struct Axis1Params {
    float2* X;            // [M][n1][n2][cols], transformed in place along n1
    const float2* tw1;
    AxisPlan p1;
    int32_t n1, n2, cols, M, tc, ncolblk;
};

// ---------------------------------------------------------------------------- recombination
// Phase tables are float32 values computed in float64 on the host:
//   tab1[mu][i1]  = b_mu e^{2 pi i g1 r_mu1},  g1 = (g0_1 + i1)/n1
//   tab2[mu][i2]  = e^{2 pi i g2 r_mu2}
//   tabK3[mu][k3] = e^{2 pi i k3 r_mu3 / n3}
//   tabH3[c][h]   = e^{2 pi i H3 r_c3},  H3 = H3min + h
//   tabK2[mu][k2] = e^{2 pi i k2 r_mu2 / n2}          (the folded form)
struct RecombParams {
    const float2* X;
    float* out;
    const float2* tab1;
    const float2* tab2;
    const float2* tabK3;
    const float2* tabH3;
    const float2* tabK2;
    int32_t n1, n2, n3, nh, S, SF, F, M, first_mono;
    int32_t g0[3], cnt[3];
    int32_t opitch, ooff;   // output element (i1, i2, i3) at out[(i1 cnt1 + i2) opitch + i3 + ooff]
    int32_t ostream;        // rows start 128-byte lines: direct writes are streaming stores
    int32_t H3min, nH3span;
    int32_t nclass;         // r3 classes (rows of tabH3)
    const int4* work;       // [nwork] (k1, k2, G1, h2a | h2b << 12 | mirror << 24), or k1 < 0;
                            // the folded form adds hasb << 25 | mirror_b << 26 | slice << 27
    int32_t nwork;
    int32_t nchunk3;        // H3 chunks per (H2, k3)
    int32_t variant;        // kernel variant (0: default for the problem, 1: multi-configuration
                            // form, 2: class form even when the parity form applies,
                            // 3: unfolded even when the folded form applies, 4: folded
                            // without k3 slices, 5: direct, order 0 only)
    int32_t fold;           // folded form: every r_mu2 is a multiple of 1/2, so the g2 phase of a
                            // site is e^{2 pi i k2 r_mu2 / n2} times +-1 by the parity of H2, and
                            // level A sums the sites of each r3 class (per H2 residue)
    int32_t fold_l2;        // H2 residues of the folded form: 1 (every r_mu2 whole) or 2
    int32_t n3s;            // folded form: k3 per slice; block slice s covers k3 in [s n3s, (s + 1) n3s)
    const int2* k3tab;      // folded form: [n3] (H3lo, count) of the H3 with k3 + n3 H3 in the box
    int32_t hmin_s[8];      // folded form, per slice: the fewest H3 values any item of a full wave has
    int32_t sgn2[kMaxSites];         // per sorted position: e^{2 pi i r_mu2} = +-1
    int32_t parity;         // every r_mu3 is a multiple of 1/2 (the parity form applies)
    int32_t nuc_ff;         // nuclear sites with |Q|-dependent scattering factors ff (class form)
    int32_t class_sign[kMaxSites];   // per class: e^{2 pi i r_c3} = +-1 in the parity form
    int32_t nsc;            // site chunks (each fits the LDS budget)
    int32_t bs_elems;       // float2 elements of the level-A buffer (the staging area follows)
    int32_t xs_elems;       // float2 elements of the staging area (the class phases follow)
    int32_t sc_start[kMaxSites + 1];   // site chunk boundaries in the sorted site list
    int32_t site_of[kMaxSites];        // sorted position -> site index
    int32_t class_of[kMaxSites];       // sorted position -> class index
    double tw[3];           // 2 pi / n_a
    float scale;            // 1/(N M)  (magnetic: C/(N M))
    // magnetic only
    float recip[9];         // rows a*, b*, c* (inverse Angstrom)
    int32_t ff_uniform;     // 1 when every site has the same form factor
    int32_t ff_sep;         // 1 when, besides, b* is orthogonal to a* and c*: |Q|^2 is then a
                            // part of (g1, g3) plus a part of g2, and each Gaussian of the form
                            // factor a product of the two parts' exponentials
    float ff[kMaxSites][8];  // per sorted position: form factor (7), unused
    // Debye-Waller factor T_mu(G) of magnetic sites with displacements: dwc[mu][t] the
    // mean over occupied atoms and configurations of u1^p u2^q u3^r (monomial t,
    // mono_index order), float64; null or dw_order 0: T = 1.  The kernel contracts p per
    // block into LDS (dw_elems float2 after the class phases), q per thread and r per voxel.
    const double* dwc;
    int32_t dw_order, dwT, dw_elems;
    // row-staged magnetic form: class c holds the sorted positions
    // [class_start[c], class_start[c + 1]); the work list's blocks take at most
    // `rows` rows; site chunks of `csites` sites
    int32_t class_start[kMaxSites + 1];
    int32_t rows, csites;
    int32_t qmod;           // > 0: every r_c3 a multiple of 1/qmod and one form factor for all
                            // sites: the classes are summed per residue of H3 mod qmod
    int32_t qmod2;          // > 0: every r_mu2 a multiple of 1/qmod2: rows whose H2 agree mod
                            // qmod2 have the same site phases, so levels B and the residue sums
                            // run on the first min(rows, qmod2) rows of a block only
    int32_t qmod1;          // > 0: every r_mu1 a multiple of 1/qmod1: G1 planes of one column whose
                            // H1 agree mod qmod1 have the same site phases; a work item then
                            // covers 1 + ((w >> 28) & 3) planes G1 + p qmod1 n1, plane p mirrored
                            // when bit 24 + p of w is set (one configuration only)
    int32_t planes;         // direct form: the planes i1 < planes are computed (a half-stored
                            // box holds its planes G1 <= 0 only)
};

// ---------------------------------------------------------------------------- Bragg (k = 0)
struct BraggParams {
    const double* sums;     // [M*S][T]
    float* out;             // output box
    int32_t g0[3], cnt[3];
    int32_t opitch, ooff;   // output element (i1, i2, i3) at out[(i1 cnt1 + i2) opitch + i3 + ooff]
    int32_t n[3];
    int32_t Hlo[3], nH[3];  // H with n H inside the box
    int32_t S, T, M, kind;
    double scale;           // 1/N  (magnetic: C/N); the means over configurations are explicit
    const double* site;     // [S][12]: r_mu (3), b_mu, form factor (7), unused
    double recip[9];
    int32_t has_ff;
    int8_t mono[3 * kMaxMono];   // exponents (p, q, r) of monomial t (nuclear sums, or the
                                 // Debye-Waller means of a magnetic model)
    const double* dwc;      // magnetic: [S][dwT] Debye-Waller means, or null (T = 1)
    int32_t dwT;
};

// ---------------------------------------------------------------------------- Lanczos
struct LanczosParams {
    const float* in;        // I on the grown box [e1][e2][e3], rows of ipitch from ioff
    int32_t ipitch, ioff;
    int32_t ihalf;          // planes stored; plane e1 >= ihalf is read as the mirror of plane
                            // e[0] - 1 - e1 (I(-G) = I(G) on a symmetric box)
    int32_t ohalf;          // 0, or the output planes computed on a symmetric output box: each
                            // is also written mirrored (the filter commutes with G -> -G)
    float* out;             // [o1][o2][o3]
    const float* wn;        // [s][2m] normalised weights (the same on every axis)
    int32_t e[3], o[3];
    int32_t m, s;
    int32_t eoff;           // input index of the first window point of output 0
    int32_t t1, t2, t3;     // tile extents (outputs)
    int32_t nb1, nb2, nb3;
};

// Windowed-sinc sum at arbitrary points Q (one thread per point): I(G) on the box
// [e0, e0 + e) of every window, G_a in [floor(Q_a) - w + 1, floor(Q_a) + w].
constexpr int kPointsMaxHalfwidth = 8;
struct PointsParams {
    const float* in;        // I(G) [e1][e2][e3], dense
    const double* q;        // [npts][3] points in units of the supercell Bragg grid
    float* out;             // [npts]
    int64_t npts;
    int32_t e0[3], e[3];
    int32_t w;              // window half-width m m'/2 (<= kPointsMaxHalfwidth)
    float rcut;             // (1 - 1/m)/m'
};

// ---------------------------------------------------------------------------- merged launches
// Several launches of one kernel (one per model of a batch) can run as one grid: the
// launch of descriptor d, g_d blocks, takes the merged blocks [first_d, first_d + g_d),
// first_d a multiple of 8, so a block sits on the XCD it would have in its own launch
// (the dispatcher deals consecutive blocks round-robin to the 8 XCDs) and the kernels'
// XCD-aware tile orders still hold.  Each group of 8 merged blocks has one slot.
struct Slot {
    int32_t d;              // descriptor: index into the kernel's parameter array
    int32_t first;          // first merged block of the descriptor
    int32_t count;          // blocks of the descriptor's own launch
    int32_t pad;
};

// Descriptor and block index (within its own launch) of this block; false on the
// padding blocks past the descriptor's own grid.
// A pointer taken from a descriptor table is generic to the compiler (flat memory
// operations, which also hold the scalar-load counter); a kernel body reads and writes its
// device buffers through this global-address-space view instead.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// p[i] of a complex array through the global view (one 8-byte load)
__device__ __forceinline__ float2 ldg2(const float2* p, size_t i)
{
    return __builtin_bit_cast(float2, ((const __attribute__((address_space(1))) unsigned long long*)p)[i]);
}

// p[i] = v for a complex array through the global view (one 8-byte store)
__device__ __forceinline__ void stg2(float2* p, size_t i, float2 v)
{
    ((__attribute__((address_space(1))) unsigned long long*)p)[i] = __builtin_bit_cast(unsigned long long, v);
}

__device__ __forceinline__ bool slot_of(const Slot* __restrict__ slots, int& d, int& bx)
{
    const Slot s = slots[blockIdx.x >> 3];
    d = s.d;
    bx = (int)blockIdx.x - s.first;
    return bx < s.count;
}

// One launch as recorded for a merged batch: the merged form of its kernel, its grid,
// block and dynamic LDS, and a copy of its parameter block.
struct LaunchRec {
    const void* one = nullptr;      // kernel (P params)
    const void* merged = nullptr;   // kernel (const P* params, const Slot* slots)
    uint32_t grid = 0, block = 0, lds = 0;
    const char* stage = "";         // the step of the path it belongs to
    std::vector<unsigned char> params;
};

// While a host thread's recorder is set, the launchers append their launches to it
// instead of issuing them (the batch planner reads the sequence of each model).
struct Recorder {
    std::vector<LaunchRec> recs;
    const char* stage = "";
};
inline thread_local Recorder* g_recorder = nullptr;

// Issue a launch of `one` (or record it with its merged form `merged`).
template <class P>
hipError_t dispatch(void (*one)(P), void (*merged)(const P*, const Slot*), unsigned grid, unsigned block,
                    size_t lds, hipStream_t st, const P& p)
{
    if (grid == 0) return hipSuccess;
    if (Recorder* r = g_recorder) {
        LaunchRec rec;
        rec.one = reinterpret_cast<const void*>(one);
        rec.merged = reinterpret_cast<const void*>(merged);
        rec.grid = grid; rec.block = block; rec.lds = (uint32_t)lds;
        rec.stage = r->stage;
        rec.params.resize(sizeof(P));
        __builtin_memcpy(rec.params.data(), &p, sizeof(P));
        r->recs.push_back(std::move(rec));
        return hipSuccess;
    }
    void* args[] = {const_cast<P*>(&p)};
    return hipLaunchKernel(reinterpret_cast<const void*>(one), dim3(grid), dim3(block), args, lds, st);
}

// ---------------------------------------------------------------------------- launchers
hipError_t launch_sums(const SumsParams& p, int order, hipStream_t st);
hipError_t launch_fft_planes(const PlaneParams& p, hipStream_t st);
hipError_t launch_fft_axis1(const Axis1Params& p, hipStream_t st);
hipError_t launch_recombine_nuclear(const RecombParams& p, int order, int hc, int block,
                                    size_t lds, hipStream_t st);
hipError_t launch_recombine_magnetic(const RecombParams& p, int hc, int block, size_t lds,
                                     hipStream_t st);
// the direct form (Taylor order 0, one field per site): one thread per voxel of the box
hipError_t launch_recombine_direct(const RecombParams& p, hipStream_t st);
// the row-staged magnetic form (no Debye-Waller factor); p.work lists its blocks, and
// the launch has one thread per G3 of the box (block >= cnt3)
constexpr int kMagRowsMaxThreads = 512;
constexpr int kMagRowsMaxRows = 16;
constexpr int kMagRowsMaxClasses = 8;   // the per-residue class sums need q <= nclass <= this
hipError_t launch_recombine_magnetic_rows(const RecombParams& p, int block, size_t lds, hipStream_t st);
// float2 elements of its LDS for `rows` staged rows (a block's rows, or min(rows, qmod2)),
// site chunks of csites, S sites, nclass classes
inline size_t magnetic_rows_lds_elems(int rows, int csites, int S, int nclass, int n3, int nH3span)
{
    return (size_t)rows * nclass * 3 * n3 + (size_t)S * n3 + (size_t)rows * S + (size_t)nclass * nH3span
         + (size_t)csites * 3 * n3;
}
hipError_t launch_bragg(const BraggParams& p, int order, hipStream_t st);
// dwc[mu][t] = sum_m sums[m][mu][t] / sum_m sums[m][mu][0] (0 for a site with no atom):
// the Debye-Waller means of Eq. dw from the float64 lattice sums of the displacements.
struct DwParams {
    const double* sums;     // [M][S][T]
    double* dwc;            // [S][T]
    int32_t M, S, T;
};
hipError_t launch_dw_mean(const DwParams& p, hipStream_t st);
hipError_t launch_lanczos(const LanczosParams& p, hipStream_t st);
hipError_t launch_lanczos_points(const PointsParams& p, hipStream_t st);
// the spherical cutoff: p.wn holds [s^3][(2m)^3] normalised weights; m in {2, 3, 4}
hipError_t launch_lanczos_stencil(const LanczosParams& p, hipStream_t st);

// Block sizes / LDS limits the host planner must respect.
int recombine_max_threads(int hc, int magnetic);
size_t planes_lds_bytes(const PlaneParams& p);
size_t axis1_lds_bytes(const Axis1Params& p);
size_t lanczos_lds_bytes(const LanczosParams& p);

}  // namespace dsx
