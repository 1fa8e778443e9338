// Reciprocal-space recombination of the per-site spectra into the diffuse
// intensity at every supercell Bragg point G of a box, for gfx950.
//
// For G = H + k (Sec. III, Eq. g_vec; k = G mod n) the structure factor of one
// configuration is (Sec. III.C, Eq. total_sf_taylor, regrouped by monomial)
//
//   F(G) = sum_mu b_mu e^{2 pi i g.r_mu} sum_{p+q+r<=N}
//          (i t1)^p/p! (i t2)^q/q! (i t3)^r/r! X^{pqr}_mu(k),   t_a = 2 pi g_a,
//
// with X the +i FFT of delta u1^p u2^q u3^r.  It is evaluated by sum factorisation
// over the three axes:
//   level A (per block: fixed k1, k2 and H1, i.e. fixed g1)
//       B_mu^{qr}(k3) = b_mu e^{2 pi i g1 r_mu1} sum_p (i t1)^p/p! X^{pqr}_mu(k1,k2,k3)
//       in LDS; the spectra of one site of column (k1, k2), then of the mirrored
//       column (-k1, -k2) that supplies k3 > n3/2 through X(k) = conj X(-k), are
//       staged in LDS with independent coalesced loads;
//   level B (per thread: fixed H2 and k3)
//       D_c^r = sum_{mu in c} e^{2 pi i (g2 r_mu2 + k3 r_mu3/n3)} sum_q (i t2)^q/q! B_mu^{qr} / r!
//       where the class c groups the sites that share r_mu3;
//   level C (per voxel: the thread's H3 values)
//       F = sum_c e^{2 pi i H3 r_c3} sum_r (i t3)^r D_c^r   (Horner in i t3),
// then |F|^2 is accumulated over the configurations in registers and written
// once, with consecutive lanes writing consecutive G3.  The magnetic kernel uses
// the three spin-component spectra instead of the Taylor monomials, applies the
// form factor and takes the component of F perpendicular to Q (Sec. III.D,
// Eqs. mag_sf, mag_intensity, mag_projection).
//
// Folded form: when every r_mu2 is a multiple of 1/2, e^{2 pi i g2 r_mu2} =
// e^{2 pi i k2 r_mu2 / n2} (+-1)^{H2}, so the g2 phase splits into a block-uniform
// factor and a sign fixed by the parity of H2.  Level A then applies the site's whole
// phase but that sign (and 1/r!), and sums the sites of each r3 class into one buffer
// per H2 parity; level B contracts q once per class instead of once per site.
//
// Blocks walk a host-built work list of (k1, k2, G1, H2 range) items, already in
// the order that keeps the blocks of one column (and of its mirror) on one XCD.
// On a box symmetric about G = 0 the list holds only half of the G1 planes and the
// blocks also write I(-G) = I(G) (Friedel symmetry, exact for real fields and for
// the truncated Taylor series).
//
// The points k = 0 (G = 0 mod n) are computed separately in float64 from the
// float64 lattice sums (k_bragg_*), where the Bragg subtraction |<F>|^2 cancels
// most of |F|^2 (Sec. II, Eq. bragg_diffuse_sf; Sec. III.A, Eq. bragg_sf); the
// ensemble mean <F> is the mean over the model's configurations.
#include <type_traits>

#include "dsx_internal.h"

namespace dsx {

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ int floordiv(int a, int b) {   // b > 0
    int q = a / b;
    if ((a % b) != 0 && (a < 0)) --q;
    return q;
}
__device__ __forceinline__ int ceildiv(int a, int b) { return -floordiv(-a, b); }
// H values of residue k on one axis: lo, count with g0 <= k + n H < g0 + cnt
__device__ __forceinline__ void hrange(int k, int n, int g0, int cnt, int& lo, int& count) {
    lo = ceildiv(g0 - k, n);
    const int hi = floordiv(g0 + cnt - 1 - k, n);
    count = hi >= lo ? hi - lo + 1 : 0;
}

__host__ __device__ constexpr float inv_factorial(int r) {
    float f = 1.f;
    for (int i = 2; i <= r; ++i) f *= (float)i;
    return 1.f / f;
}

// 1/r! for a run-time r <= kMaxOrder.
__device__ __forceinline__ float inv_factorial_rt(int r)
{
    float v = 1.f;
#pragma unroll
    for (int i = 2; i <= kMaxOrder; ++i) v = (r == i) ? inv_factorial(i) : v;
    return v;
}

// Quotient a / b for 0 <= a < 2^22 and 0 < b < 2^22, with rb ~= 1/b (float): the
// float estimate is off by at most one and is corrected with one remainder check.
__device__ __forceinline__ int qdiv_r(int a, int b, float rb)
{
    int q = (int)((float)a * rb);
    const int r = a - q * b;
    q += (r >= b) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

// Cooperative global -> LDS copy with up to eight independent loads in flight per
// thread before any of them is stored.
__device__ __forceinline__ void stage_copy(float2* __restrict__ dst, const float2* __restrict__ src,
                                           int total)
{
    for (int base = threadIdx.x; base < total; base += 8 * blockDim.x) {
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * blockDim.x;
            if (i < total) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * blockDim.x;
            if (i < total) dst[i] = v[u];
        }
    }
}

struct BlockWork {
    int k1, k2, G1, i1, h2a, h2b, H2lo;
    bool mirror;
};

__device__ __forceinline__ bool decode_block(const RecombParams& P, BlockWork& w, const int bx)
{
    const int4 it = P.work[bx];
    if (it.x < 0) return false;
    w.k1 = it.x;
    w.k2 = it.y;
    w.G1 = it.z;
    w.h2a = it.w & 0xfff;
    w.h2b = (it.w >> 12) & 0xfff;
    w.mirror = (it.w >> 24) & 1;
    int nH2;
    hrange(w.k2, P.n2, P.g0[1], P.cnt[1], w.H2lo, nH2);
    w.i1 = w.G1 - P.g0[0];
    return true;
}

// Copy the class phase table e^{2 pi i H3 r_c3} into LDS; returns the pointer to
// index with an absolute H3.
__device__ __forceinline__ const float2* stage_class_phases(const RecombParams& P, float2* dst)
{
    const int tot = P.nclass * P.nH3span;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) dst[i] = P.tabH3[i];
    return dst - P.H3min;
}

// Word 3 of a raw buffer resource on gfx9-class targets: 32-bit data format (a zero
// format would read zeros); no swizzle, stride 0, so offsets are plain byte offsets
// checked against the record count.
constexpr int kBufferFlags = 0x00020000;
constexpr uint32_t kNoRecord = 0x80000000u;   // an offset past every record count used here

// f(s) of a site: the analytic form factor A e^{-a s^2} + B e^{-b s^2} + C e^{-c s^2} + D.
// Magnetic sites use it as f_mag of Eq. mag_sf, nuclear sites as a |Q|-dependent
// scattering factor.
__device__ __forceinline__ float site_ff(const float* f, float s2) {
    return f[0] * expf(-f[1] * s2) + f[2] * expf(-f[3] * s2) + f[4] * expf(-f[5] * s2) + f[6];
}

// ---------------------------------------------------------------------------- nuclear
__device__ __forceinline__ int wave_min_uniform(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// The thread's output voxels G3 = G3(h = 0) + n3 h of row (G1, G2) and, on symmetric
// boxes, their mirrors -G: byte offsets from block-uniform plane bases (a plane of
// the box is below 4 GiB), so each store is one 32-bit add and a global store.
struct RowOut {
    __attribute__((address_space(1))) char* oplane;
    __attribute__((address_space(1))) char* mplane;
    uint32_t o0, m0, step;
    bool nt;
    // On line-aligned rows every H3 step of a row is whole lines: streaming stores
    // keep the output (not read again here) out of L2, where the spectra columns stay.
    // Unaligned rows go through L2, which merges the partial lines.
    __device__ __forceinline__ void put(int h, float v) const {
        auto* a = reinterpret_cast<__attribute__((address_space(1))) float*>(oplane + (o0 + step * (uint32_t)h));
        if (nt) __builtin_nontemporal_store(v, a);
        else *a = v;
    }
    __device__ __forceinline__ void put_mirror(int h, float v) const {
        auto* a = reinterpret_cast<__attribute__((address_space(1))) float*>(mplane + (m0 - step * (uint32_t)h));
        if (nt) __builtin_nontemporal_store(v, a);
        else *a = v;
    }
};

__device__ __forceinline__ RowOut row_out(const RecombParams& P, const BlockWork& w, int i2, int i3b)
{
    RowOut r;
    const size_t plane = (size_t)P.cnt[1] * P.opitch;
    r.oplane = reinterpret_cast<__attribute__((address_space(1))) char*>(gptr(P.out) + P.ooff + (size_t)w.i1 * plane);
    r.mplane = reinterpret_cast<__attribute__((address_space(1))) char*>(gptr(P.out) + P.ooff + (size_t)(P.cnt[0] - 1 - w.i1) * plane);
    r.o0 = 4u * (uint32_t)(i2 * P.opitch + i3b);
    r.m0 = 4u * (uint32_t)((P.cnt[1] - 1 - i2) * P.opitch + (P.cnt[2] - 1 - i3b));
    r.step = 4u * (uint32_t)P.n3;
    r.nt = P.ostream != 0;
    return r;
}

// Writes v(h) for the thread's H3 values: unconditionally while every lane of the
// wave has it (h < hmin and the whole wave active), with a per-lane test otherwise.
template <int HC, bool MIRROR, typename Val>
__device__ __forceinline__ void write_row(const RowOut& ro, bool full, bool active, int hmin, int hcnt,
                                          float scale, Val val)
{
#pragma unroll
    for (int h = 0; h < HC; ++h) {
        if (h < hmin && full) {
            const float v = val(h) * scale;
            ro.put(h, v);
            if (MIRROR) ro.put_mirror(h, v);
        } else if (active && h < hcnt) {
            const float v = val(h) * scale;
            ro.put(h, v);
            if (MIRROR) ro.put_mirror(h, v);
        }
    }
}

// Level C in the parity form: the coefficient set of even H3 goes to DE and that of
// odd H3 to DO (h0 = H3 of h = 0) ...
template <int N>
__device__ __forceinline__ void parity_order(float2 (&DE)[N + 1], float2 (&DO)[N + 1], int h0)
{
    const bool odd0 = (h0 & 1) != 0;
#pragma unroll
    for (int r = 0; r <= N; ++r) {
        const float2 t = DE[r];
        DE[r] = odd0 ? DO[r] : DE[r];
        DO[r] = odd0 ? t : DO[r];
    }
}

// ... and |sum_r (i t3)^r S_r|^2 at the thread's h (Horner in i t3).
template <int N>
__device__ __forceinline__ float parity_eval(const float2 (&S)[N + 1], float t3)
{
    float2 acc = S[N];
#pragma unroll
    for (int r = N - 1; r >= 0; --r)
        acc = make_float2(S[r].x - t3 * acc.y, S[r].y + t3 * acc.x);
    return acc.x * acc.x + acc.y * acc.y;
}

// MULTI: more than one configuration; a single configuration needs no separate
// |F|^2 accumulator, and the registers it frees hold the level-A prefetch.
// PAR: every r_mu3 is a multiple of 1/2, so e^{2 pi i H3 r_c3} = +-1 by the parity
// of H3: level B folds the classes into two coefficient sets, one for even and one
// for odd H3, and level C evaluates a single polynomial per voxel.
template <int N, int HC, bool MULTI, bool PAR, class PT>
__device__ __forceinline__ void recombine_nuclear_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    constexpr int QR = n_pairs(N);
    BlockWork w;
    if (!decode_block(P, w, bx)) return;
    float2* Bs = smem;                                  // [sites of the chunk][n3][QR]
    float2* Xs = smem + P.bs_elems;                     // [F][nh] staging
    float2* tHs = Xs + P.xs_elems;                      // [nclass][nH3span]
    __shared__ int jtab[2][QR];                         // e = q + r and first field of pair j
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3, nh = P.nh;
    const int SFnh = P.SF * nh;
    const float tau1 = (float)(6.283185307179586 * (double)w.G1 / (double)n1);
    for (int j = threadIdx.x; j < QR; j += blockDim.x) {
        int e = 0;
        while ((e + 1) * (e + 2) / 2 <= j) ++e;
        int cum = 0;
        for (int ee = 0; ee < e; ++ee) cum += (ee + 1) * (N - ee + 1);
        cum += (j - e * (e + 1) / 2) * (N - e + 1);
        jtab[0][j] = e;
        jtab[1][j] = cum - P.first_mono;
    }
    const float2* tH0 = PAR ? nullptr : stage_class_phases(P, tHs);

    // this thread's item: (H2, H3 chunk, k3) with k3 fastest
    const int nitems = (w.h2b - w.h2a) * n3 * P.nchunk3;
    const int item = threadIdx.x;
    const bool active = item < nitems;
    int k3 = 0, ch = 0, h2 = w.h2a;
    if (active) {
        k3 = item % n3;
        const int r = item / n3;
        ch = r % P.nchunk3;
        h2 = w.h2a + r / P.nchunk3;
    }
    const int G2 = w.k2 + n2 * (w.H2lo + h2);
    const int i2 = G2 - P.g0[1];
    int H3lo, nH3;
    hrange(k3, n3, P.g0[2], P.cnt[2], H3lo, nH3);
    const int hbeg = ch * HC;
    const int hcnt = active ? max(0, min(HC, nH3 - hbeg)) : 0;
    const int hmin = wave_min_uniform(active ? hcnt : HC);   // iterations every lane needs
    const float tau2 = (float)(6.283185307179586 * (double)G2 / (double)n2);
    const float c3 = (float)(6.283185307179586 / (double)n3);
    const float t3base = (float)(k3 + n3 * (H3lo + hbeg)) * c3;   // tau3 of h = 0
    const float dt3 = 6.283185307179586f;                          // tau3 step per H3
    float a2[N + 1];   // tau2^q / q!
    a2[0] = 1.f;
#pragma unroll
    for (int q = 1; q <= N; ++q) a2[q] = a2[q - 1] * tau2 / (float)q;
    // g1 a* + g2 b* of the thread's row (for |Q|-dependent scattering factors)
    const float g1f = (float)w.G1 / (float)n1, g2f = (float)G2 / (float)n2;
    const float q12x = g1f * P.recip[0] + g2f * P.recip[3];
    const float q12y = g1f * P.recip[1] + g2f * P.recip[4];
    const float q12z = g1f * P.recip[2] + g2f * P.recip[5];

    float I[MULTI ? HC : 1];
#pragma unroll
    for (int h = 0; h < (MULTI ? HC : 1); ++h) I[h] = 0.f;

    const size_t col = ((size_t)w.k1 * n2 + w.k2) * SFnh;
    const size_t colm = ((size_t)((n1 - w.k1) % n1) * n2 + (n2 - w.k2) % n2) * SFnh;

    constexpr int NF = PAR ? 1 : HC;
    float2 F[NF];           // class mode: F(H3) accumulated over the classes
    float2 DE[N + 1], DO[N + 1];   // parity mode: coefficient sets of even / odd H3
    for (int m = 0; m < P.M; ++m) {
#pragma unroll
        for (int h = 0; h < NF; ++h) F[h] = make_float2(0.f, 0.f);
#pragma unroll
        for (int r = 0; r <= N; ++r) { DE[r] = make_float2(0.f, 0.f); DO[r] = make_float2(0.f, 0.f); }
        const float2* Xm = P.X + (size_t)m * n1 * n2 * SFnh;
        for (int sc = 0; sc < P.nsc; ++sc) {
            const int s0 = P.sc_start[sc], s1 = P.sc_start[sc + 1];
            const int ns = s1 - s0;
            // level A: stages (site, half); the next stage's spectra are loaded into
            // registers while the current stage is contracted from LDS
            const int nhalf = (n3 - nh > 0) ? 2 : 1;
            const int nst = ns * nhalf;
            const int stot = P.F * nh;
            constexpr int PF = (MULTI || (PAR && N >= 6)) ? 1 : 6;
            float2 pf[PF];
            auto stage_src = [&](int st) {
                const int mu = P.site_of[s0 + st / nhalf];
                return Xm + ((st % nhalf) ? colm : col) + (size_t)mu * P.F * nh;
            };
            auto prefetch = [&](const float2* src) {
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int i = threadIdx.x + u * blockDim.x;
                    if (i < stot) pf[u] = src[i];
                }
            };
            prefetch(stage_src(0));
            for (int st = 0; st < nst; ++st) {
                const int sl = st / nhalf, half = st % nhalf;
                const int mu = P.site_of[s0 + sl];
                const float2 wbase = P.tab1[(size_t)mu * P.cnt[0] + w.i1];
                const int k3lo = half ? nh : 0;
                const int nk = half ? n3 - nh : nh;
                __syncthreads();
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int i = threadIdx.x + u * blockDim.x;
                    if (i < stot) Xs[i] = pf[u];
                }
                if (stot > PF * (int)blockDim.x)       // large spectra: the rest in batches
                    stage_copy(Xs + PF * blockDim.x, stage_src(st) + PF * blockDim.x, stot - PF * blockDim.x);
                if (st + 1 < nst) prefetch(stage_src(st + 1));
                __syncthreads();
                const float sg = half ? -1.f : 1.f;
                for (int idx = threadIdx.x; idx < QR * nk; idx += blockDim.x) {
                    const int j = idx / nk;
                    const int kk = k3lo + (idx - j * nk);
                    const int e = jtab[0][j];
                    const int f0 = jtab[1][j];           // field of p = 0 (may be -1)
                    const float2* xs = Xs + f0 * nh + (half ? n3 - kk : kk);
                    // sum_p wbase (i tau1)^p / p! x_p = wbase (E + i O): E, O sum the even and odd
                    // p-terms with the real weights tau1^p / p! times the sign of i^p's nonzero
                    // part; the mirror sign of x's imaginary part is applied to the sums
                    float2 E = make_float2(0.f, 0.f), O = E;
                    float mag = 1.f;
#pragma unroll
                    for (int p = 0; p <= N; ++p) {
                        if (p <= N - e) {
                            if (f0 + p >= 0) {
                                const float2 x = xs[p * nh];
                                const float c = ((p & 3) < 2) ? mag : -mag;
                                if (p & 1) { O.x = fmaf(c, x.x, O.x); O.y = fmaf(c, x.y, O.y); }
                                else { E.x = fmaf(c, x.x, E.x); E.y = fmaf(c, x.y, E.y); }
                            }
                            mag *= tau1 * (1.f / (float)(p + 1));
                        }
                    }
                    E.y *= sg;
                    O.y *= sg;
                    Bs[((size_t)sl * n3 + kk) * QR + j] = cmulf(wbase, make_float2(E.x - O.y, E.y + O.x));
                }
            }
            __syncthreads();
            // level B (+ level C in class mode)
            if (active) {
                int sp = s0;
                while (sp < s1) {
                    const int c = P.class_of[sp];
                    int se = sp + 1;
                    while (se < s1 && P.class_of[se] == c) ++se;
                    float2 D[PAR ? 1 : N + 1];
                    if constexpr (!PAR) {
#pragma unroll
                        for (int r = 0; r <= N; ++r) D[r] = make_float2(0.f, 0.f);
                    }
                    const float sgn_odd = PAR ? (float)P.class_sign[c] : 1.f;
                    for (int sl = sp - s0; sl < se - s0; ++sl) {
                        const int mu = P.site_of[s0 + sl];
                        const float2 ph = cmulf(P.tab2[(size_t)mu * P.cnt[1] + i2],
                                                P.tabK3[(size_t)mu * n3 + k3]);
                        const float2* Bp = Bs + ((size_t)sl * n3 + k3) * QR;
#pragma unroll
                        for (int r = 0; r <= N; ++r) {
                            float2 C = make_float2(0.f, 0.f);
#pragma unroll
                            for (int q = 0; q + r <= N; ++q) {
                                const float2 v = Bp[pair_index(q, r)];
                                const float a = a2[q];
                                // C += i^q a v
                                if ((q & 3) == 0) { C.x += a * v.x; C.y += a * v.y; }
                                else if ((q & 3) == 1) { C.x -= a * v.y; C.y += a * v.x; }
                                else if ((q & 3) == 2) { C.x -= a * v.x; C.y -= a * v.y; }
                                else { C.x += a * v.y; C.y -= a * v.x; }
                            }
                            const float2 pc = cmulf(ph, C);
                            if constexpr (PAR) {
                                DE[r].x += pc.x * inv_factorial(r);
                                DE[r].y += pc.y * inv_factorial(r);
                                DO[r].x += sgn_odd * pc.x * inv_factorial(r);
                                DO[r].y += sgn_odd * pc.y * inv_factorial(r);
                            } else {
                                D[r].x += pc.x * inv_factorial(r);
                                D[r].y += pc.y * inv_factorial(r);
                            }
                            // keep the coefficient loads of one r at a time in registers
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    if constexpr (!PAR) {
                        const float2* tH = tH0 + (size_t)c * P.nH3span + H3lo + hbeg;
#pragma unroll
                        for (int h = 0; h < HC; ++h) {
                            if (h < hmin || h < hcnt) {
                                const float t3 = t3base + (float)h * dt3;
                                float2 acc = D[N];
#pragma unroll
                                for (int r = N - 1; r >= 0; --r)
                                    acc = make_float2(D[r].x - t3 * acc.y, D[r].y + t3 * acc.x);
                                float2 e3 = tH[h];
                                if (P.nuc_ff) {
                                    // the class's scattering factor f(|Q|), s = |Q|/(4 pi)
                                    const float g3 = (float)(k3 + n3 * (H3lo + hbeg + h)) / (float)n3;
                                    const float qx = q12x + g3 * P.recip[6], qy = q12y + g3 * P.recip[7],
                                                qz = q12z + g3 * P.recip[8];
                                    const float f = site_ff(P.ff[sp], (qx * qx + qy * qy + qz * qz) * 0.00633257397764611f);
                                    e3 = make_float2(e3.x * f, e3.y * f);
                                }
                                F[h].x += e3.x * acc.x - e3.y * acc.y;
                                F[h].y += e3.x * acc.y + e3.y * acc.x;
                            }
                        }
                    }
                    sp = se;
                }
            }
        }
        if constexpr (PAR && MULTI) {
            parity_order<N>(DE, DO, H3lo + hbeg);
#pragma unroll
            for (int h = 0; h < HC; ++h)
                if (h < hmin || h < hcnt) I[h] += parity_eval<N>((h & 1) ? DO : DE, t3base + (float)h * dt3);
        } else if constexpr (MULTI) {
#pragma unroll
            for (int h = 0; h < HC; ++h) I[h] += F[h].x * F[h].x + F[h].y * F[h].y;
        }
    }
    const int i3b = k3 + n3 * (H3lo + hbeg) - P.g0[2];       // output index of h = 0
    const RowOut ro = row_out(P, w, i2, i3b);
    const bool full = wave_min_uniform(active ? 1 : 0) != 0;
    if constexpr (PAR && !MULTI) parity_order<N>(DE, DO, H3lo + hbeg);
    auto val = [&](int h) -> float {
        if constexpr (MULTI) return I[h];
        else if constexpr (PAR) return parity_eval<N>((h & 1) ? DO : DE, t3base + (float)h * dt3);
        else return F[h].x * F[h].x + F[h].y * F[h].y;
    };
    if (w.mirror) write_row<HC, true>(ro, full, active, hmin, hcnt, P.scale, val);
    else write_row<HC, false>(ro, full, active, hmin, hcnt, P.scale, val);
}

template <int N, int HC, bool MULTI, bool PAR>
__global__ __launch_bounds__(512, 4) void k_recombine_nuclear(RecombParams P) { recombine_nuclear_body<N, HC, MULTI, PAR, RecombParams>(P, blockIdx.x); }
template <int N, int HC, bool MULTI, bool PAR>
__global__ __launch_bounds__(512, 4) void k_recombine_nuclear_merged(const RecombParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) recombine_nuclear_body<N, HC, MULTI, PAR, const RecombParams&>(tab[d], bx);
}

// Folded form (every r_mu2 a multiple of 1/2; see the top of the file).  A block
// takes two planes G1 and G1 + n1 of one spectra column (the second may be absent)
// and one slice of n3s k3 values: level A reads every spectrum of the slice once for
// both planes, and each half of the block then runs levels B and C of one plane.
// Slicing k3 keeps the LDS of a block small enough for two blocks per CU, so the
// load-bound level A of one overlaps the arithmetic and stores of the other.  LDS:
//   Bs   [2][nclass][L2][n3s][QR] level A summed over the sites of each r3 class,
//                                 with the site phase (but the H2-parity sign) and 1/r!
//   wt   [2][2][S][N + 1]         level-A weights (conjugated copy, plane, site, p)
//   tHs  [nclass][nH3span]        class phases e^{2 pi i H3 r_c3} (class form only)
// Level A reads the spectra straight from the (L2-resident) column: every thread
// owns (pair, k3) items and accumulates the sites of a class in registers, with the
// loads of the next site in flight, so the level needs no staging and no barrier.
// One configuration in the parity form: at most 80 VGPRs, so that three 512-thread sliced
// blocks share a CU (their LDS fits too); the multi-configuration form keeps its |F|^2
// accumulators and the class form its per-H3 structure factors in registers.
template <int N, int HC, bool MULTI, bool PAR, class PT>
__device__ __forceinline__ void recombine_folded_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    constexpr int QR = n_pairs(N);
    const int4 wi = P.work[bx];
    if (wi.x < 0) return;
    const bool hasb = (wi.w >> 25) & 1;
    const int n3s = P.n3s;
    const int k3a = ((wi.w >> 27) & 7) * n3s;       // first k3 of the slice
    const int k3n = min(n3s, P.n3 - k3a);          // k3 in the slice
    const int bh = blockDim.x >> 1;                 // threads per plane (a multiple of 64)
    // the plane of this thread's B / C item (wave-uniform: its output bases are scalars)
    const int sel = __builtin_amdgcn_readfirstlane((int)threadIdx.x >= bh ? 1 : 0);
    BlockWork w;
    w.k1 = wi.x;
    w.k2 = wi.y;
    w.G1 = wi.z + (sel && hasb ? P.n1 : 0);
    w.h2a = wi.w & 0xfff;
    w.h2b = (wi.w >> 12) & 0xfff;
    w.mirror = ((wi.w >> (sel ? 26 : 24)) & 1) != 0;
    {
        int nH2;
        hrange(w.k2, P.n2, P.g0[1], P.cnt[1], w.H2lo, nH2);
    }
    w.i1 = w.G1 - P.g0[0];
    const int L2 = P.fold_l2;
    float2* Bs = smem + (size_t)sel * P.bs_elems;
    // per plane and site: b e^{2 pi i (g1 r1 + k2 r2 / n2)} (i tau1)^p / p!, and its
    // conjugate for the mirrored half (sum w conj(x) = conj(sum conj(w) x))
    float2* wt = smem + 2 * (size_t)P.bs_elems;
    float2* tHs = wt + 4 * P.S * (N + 1);
    __shared__ int jtab[2][QR];              // terms N - e + 1, field of p = 0 of pair j
    __shared__ float jfr[QR];                // 1/r! of pair j
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3, nh = P.nh;
    const int SFnh = P.SF * nh;
    for (int j = threadIdx.x; j < QR; j += blockDim.x) {
        int e = 0;
        while ((e + 1) * (e + 2) / 2 <= j) ++e;
        int cum = 0;
        for (int ee = 0; ee < e; ++ee) cum += (ee + 1) * (N - ee + 1);
        const int r = j - e * (e + 1) / 2;   // pair_index(q, r) = e (e + 1) / 2 + r
        cum += r * (N - e + 1);
        jtab[0][j] = N - e + 1;
        jtab[1][j] = cum - P.first_mono;
        jfr[j] = inv_factorial_rt(r);
    }
    // level-A weights w_p = b e^{2 pi i (g1 r1 + k2 r2 / n2)} (i tau1)^p / p!: per plane the real
    // c_p = sqrt(scale) tau1^p / p! with the sign of i^p's nonzero part (+ for p mod 4 in {0, 1},
    // - for {2, 3}), and per (plane, site) the phase wb, so that sum_p w_p x_p = wb (E + i O)
    // with E, O the sums of c_p x_p over even and odd p
    float* cm = reinterpret_cast<float*>(wt);                  // [2][N + 1]
    float2* wbt = wt + (N + 1);                                 // [2][S]
    for (int t = threadIdx.x; t < 2 * (N + 1); t += blockDim.x) {
        const int pl = t / (N + 1), p = t - pl * (N + 1);
        const int G1 = wi.z + (pl && hasb ? n1 : 0);      // (an absent plane repeats the first)
        const float tau1 = (float)((double)G1 * P.tw[0]);
        // sqrt(scale) here scales every |F|^2 by the output scale at no cost per voxel
        float mag = inv_factorial_rt(p) * sqrtf(P.scale);
        for (int v = 1; v <= p; ++v) mag *= tau1;
        cm[t] = ((p & 3) < 2) ? mag : -mag;
    }
    for (int t = threadIdx.x; t < 2 * P.S; t += blockDim.x) {
        const int pl = t / P.S, sl = t - pl * P.S;
        const int mu = P.site_of[sl];
        const int G1 = wi.z + (pl && hasb ? n1 : 0);
        wbt[t] = cmulf(P.tab1[(size_t)mu * P.cnt[0] + (G1 - P.g0[0])], P.tabK2[(size_t)mu * n2 + w.k2]);
    }
    const float2* tH0 = PAR ? nullptr : stage_class_phases(P, tHs);

    // this thread's item: (H2, H3 chunk, k3 of the slice) with k3 fastest, in its plane
    const int nitems = (w.h2b - w.h2a) * k3n * P.nchunk3;
    const int item = threadIdx.x - sel * bh;
    const bool active = item < nitems && (sel == 0 || hasb);
    int k3 = k3a, ch = 0, h2 = w.h2a;
    if (active) {
        const int r = qdiv_r(item, k3n, 1.f / (float)k3n);
        k3 = k3a + (item - r * k3n);
        const int rc = P.nchunk3 == 1 ? r : qdiv_r(r, P.nchunk3, 1.f / (float)P.nchunk3);
        ch = r - rc * P.nchunk3;
        h2 = w.h2a + rc;
    }
    const int H2 = w.H2lo + h2;
    const int rho = (L2 == 2) ? (H2 & 1) : 0;
    const int G2 = w.k2 + n2 * H2;
    const int i2 = G2 - P.g0[1];
    const int2 h3 = P.k3tab[k3];                   // H3 range of residue k3 in the box
    const int H3lo = h3.x, nH3 = h3.y;
    const int hbeg = ch * HC;
    const int hcnt = active ? max(0, min(HC, nH3 - hbeg)) : 0;
    const int hmin = P.hmin_s[(wi.w >> 27) & 7];   // iterations every lane of a full wave needs
    const float tau2 = (float)((double)G2 * P.tw[1]);
    const float c3 = (float)P.tw[2];
    const float t3base = (float)(k3 + n3 * (H3lo + hbeg)) * c3;   // tau3 of h = 0
    const float dt3 = 6.283185307179586f;                          // tau3 step per H3
    float I[MULTI ? HC : 1];
#pragma unroll
    for (int h = 0; h < (MULTI ? HC : 1); ++h) I[h] = 0.f;

    const size_t col = ((size_t)w.k1 * n2 + w.k2) * SFnh;
    const size_t colm = ((size_t)((n1 - w.k1) % n1) * n2 + (n2 - w.k2) % n2) * SFnh;
    const int nitemA = QR * k3n;
    const float rn3 = 1.f / (float)k3n;
    const size_t fstride = (size_t)P.F * nh;   // between the sites of a column

    constexpr int NF = PAR ? 1 : HC;
    float2 F[NF];
    float2 DE[N + 1], DO[N + 1];
    __syncthreads();
    // buffer resources: the spectra of one configuration, the k3 phase table
    const uint32_t xbytes = (uint32_t)((size_t)n1 * n2 * SFnh * sizeof(float2));
    const __amdgpu_buffer_rsrc_t rk = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float2*>(P.tabK3), (short)0, (int)(P.S * n3 * sizeof(float2)), kBufferFlags);
    // (one configuration: a constant trip count, so the coefficient sets leave no loop)
    const int nconf = MULTI ? P.M : 1;
    for (int m = 0; m < nconf; ++m) {
        const float2* Xm = P.X + (size_t)m * n1 * n2 * SFnh;
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float2*>(Xm), (short)0, (int)xbytes, kBufferFlags);
        // level A: items (pair j, k3) with k3 fastest; pairs run in order of e = q + r,
        // so the number of p terms N - e + 1 only falls along a wave: its first and
        // last lanes give the wave-uniform bounds
        for (int base = 0; base < nitemA; base += blockDim.x) {
            const int gw0 = __builtin_amdgcn_readfirstlane(base + (int)(threadIdx.x & ~63u));
            if (gw0 >= nitemA) continue;
            const int pmax = __builtin_amdgcn_readfirstlane(jtab[0][qdiv_r(gw0, k3n, rn3)]);
            const int g = base + threadIdx.x;
            const bool ok = g < nitemA;
            const int gg = ok ? g : nitemA - 1;
            const int j = qdiv_r(gg, k3n, rn3);
            const int kl = gg - j * k3n;                  // k3 within the slice
            const int kk = k3a + kl;
            const int pc = jtab[0][j], f0 = jtab[1][j];
            const float fr = jfr[j];
            const bool half = kk >= nh;                   // conj X(-k) from the mirrored column
            const unsigned cj = half ? 0x80000000u : 0u;
            // the p terms of site sl and the k3 phase of its class.  Every lane issues the
            // same N + 2 loads whatever its run length: with a fixed count in flight, the
            // wait for one site leaves the loads of the next one outstanding.  They are
            // buffer loads: per-item 32-bit byte offsets (the spectra of one configuration
            // are below 2 GiB) plus the site's offset in a scalar, so a load costs no
            // address arithmetic, and a term past the pair's run (or the absent constant
            // monomial) takes an offset past the record count and reads 0.
            const uint32_t o0 = (uint32_t)((half ? colm : col) + (size_t)(half ? n3 - kk : kk));
            uint32_t vo[N + 1];
#pragma unroll
            for (int p = 0; p <= N; ++p)
                vo[p] = (p < pc && f0 + p >= 0) ? 8u * (o0 + (uint32_t)((f0 + p) * nh)) : kNoRecord;
            const uint32_t ko = 8u * (uint32_t)kk;
            auto load = [&](int sl, float2 (&x)[N + 2]) {
                const uint32_t mu = (uint32_t)P.site_of[sl];
                const uint32_t so = mu * (uint32_t)(8 * fstride);
#pragma unroll
                for (int p = 0; p <= N; ++p)
                    x[p] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rx, vo[p], so, 0));
                x[N + 1] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rk, ko, mu * (uint32_t)(8 * n3), 0));
            };
            // ... and sum_p w_p X (X = x, or conj x on the mirrored half) for both planes:
            // wb (E + i O) from the real p-terms; the mirrored half forms sum conj(w) x =
            // conj(wb) (E - i O) and conjugates it
            const float sh = half ? -1.f : 1.f;
            auto contract = [&](int sl, const float2 (&x)[N + 2], float2& acc0, float2& acc1) {
                float2 e0 = make_float2(0.f, 0.f), o0 = e0, e1 = e0, o1 = e0;
#pragma unroll
                for (int p = 0; p <= N; ++p) {
                    if (p < pmax) {
                        const float2 v = x[p];
                        const float a = cm[p], b = cm[N + 1 + p];
                        if (p & 1) {
                            o0.x = fmaf(a, v.x, o0.x); o0.y = fmaf(a, v.y, o0.y);
                            o1.x = fmaf(b, v.x, o1.x); o1.y = fmaf(b, v.y, o1.y);
                        } else {
                            e0.x = fmaf(a, v.x, e0.x); e0.y = fmaf(a, v.y, e0.y);
                            e1.x = fmaf(b, v.x, e1.x); e1.y = fmaf(b, v.y, e1.y);
                        }
                    }
                }
                const float2 in0 = make_float2(fmaf(-sh, o0.y, e0.x), fmaf(sh, o0.x, e0.y));
                const float2 in1 = make_float2(fmaf(-sh, o1.y, e1.x), fmaf(sh, o1.x, e1.y));
                float2 w0 = wbt[sl], w1 = wbt[P.S + sl];
                w0.y *= sh;
                w1.y *= sh;
                acc0 = cmulf(w0, in0);
                acc1 = cmulf(w1, in1);
                acc0.y = __uint_as_float(__float_as_uint(acc0.y) ^ cj);
                acc1.y = __uint_as_float(__float_as_uint(acc1.y) ^ cj);
            };
            // sites in class order; the loads of the next site are in flight while the
            // current one is contracted
            float2 xa[N + 2], xb2[N + 2];
            float2 aE0 = make_float2(0.f, 0.f), aO0 = aE0, aE1 = aE0, aO1 = aE0;
            auto finish = [&](int sl, const float2 (&x)[N + 2], const float2& acc0, const float2& acc1) {
                const float s2 = (float)P.sgn2[sl];
                aE0.x += acc0.x; aE0.y += acc0.y;
                aO0.x = fmaf(s2, acc0.x, aO0.x); aO0.y = fmaf(s2, acc0.y, aO0.y);
                aE1.x += acc1.x; aE1.y += acc1.y;
                aO1.x = fmaf(s2, acc1.x, aO1.x); aO1.y = fmaf(s2, acc1.y, aO1.y);
                const int c = P.class_of[sl];
                if (sl + 1 == P.S || P.class_of[sl + 1] != c) {   // last site of class c
                    // the sites of a class share r3, hence the k3 phase: applied once, with 1/r!
                    const float2 kf = make_float2(x[N + 1].x * fr, x[N + 1].y * fr);
                    if (ok) {
                        float2* b0 = smem + ((size_t)(c * L2) * n3s + kl) * QR + j;
                        float2* b1 = b0 + P.bs_elems;
                        b0[0] = cmulf(kf, aE0);
                        b1[0] = cmulf(kf, aE1);
                        if (L2 == 2) {
                            b0[(size_t)n3s * QR] = cmulf(kf, aO0);
                            b1[(size_t)n3s * QR] = cmulf(kf, aO1);
                        }
                    }
                    aE0 = aO0 = aE1 = aO1 = make_float2(0.f, 0.f);
                }
            };
            // (the loads are unconditional: a site past the last repeats the last one)
            float2 c0, c1;
            const int slast = P.S - 1;
            load(0, xa);
            for (int sl = 0; sl < P.S; sl += 2) {
                load(min(sl + 1, slast), xb2);
                contract(sl, xa, c0, c1);
                finish(sl, xa, c0, c1);
                load(min(sl + 2, slast), xa);
                if (sl + 1 < P.S) {
                    contract(sl + 1, xb2, c0, c1);
                    finish(sl + 1, xb2, c0, c1);
                }
            }
        }
        __syncthreads();
        // level B: contract q once per class; the parity form folds the classes into
        // DE / DO, the class form evaluates level C per class
        float a2[N + 1];   // tau2^q / q!
        a2[0] = 1.f;
#pragma unroll
        for (int q = 1; q <= N; ++q) a2[q] = a2[q - 1] * tau2 * (1.f / (float)q);
#pragma unroll
        for (int h = 0; h < NF; ++h) F[h] = make_float2(0.f, 0.f);
        // (every lane: an inactive one evaluates a valid item of its block whose values are
        // never written, which keeps the wave free of merges)
        // Parity form: DE / DO are the coefficient sets of the even / odd h of the thread's
        // run (H3 = H3lo + hbeg + h), so class c enters them with e^{2 pi i H3 r_c3} =
        // sgn_c^H3 split as sgn_c^(H3lo + hbeg) (the weight wa) times sgn_c^h (wb = wa sgn_c
        // for odd h); the first class initialises the sets.
        const bool odd0 = ((H3lo + hbeg) & 1) != 0;
        auto level_b = [&](int c, auto first_tag) {
            constexpr bool FIRST = decltype(first_tag)::value;
            {
                const float2* Bp = Bs + ((size_t)(c * L2 + rho) * n3s + (k3 - k3a)) * QR;
                const float sgn = PAR ? (float)P.class_sign[c] : 1.f;
                const float wa = odd0 ? sgn : 1.f, wb = odd0 ? 1.f : sgn;
                float2 D[PAR ? 1 : N + 1];
#pragma unroll
                for (int r = 0; r <= N; ++r) {
                    float2 C = Bp[pair_index(0, r)];          // q = 0: a2[0] = 1
#pragma unroll
                    for (int q = 1; q + r <= N; ++q) {
                        const float2 v = Bp[pair_index(q, r)];
                        const float a = a2[q];
                        // C += i^q a v
                        if ((q & 3) == 0) { C.x += a * v.x; C.y += a * v.y; }
                        else if ((q & 3) == 1) { C.x -= a * v.y; C.y += a * v.x; }
                        else if ((q & 3) == 2) { C.x -= a * v.x; C.y -= a * v.y; }
                        else { C.x += a * v.y; C.y -= a * v.x; }
                    }
                    if constexpr (PAR) {
                        if constexpr (FIRST) {
                            DE[r] = make_float2(wa * C.x, wa * C.y);
                            DO[r] = make_float2(wb * C.x, wb * C.y);
                        } else {
                            DE[r].x = fmaf(wa, C.x, DE[r].x); DE[r].y = fmaf(wa, C.y, DE[r].y);
                            DO[r].x = fmaf(wb, C.x, DO[r].x); DO[r].y = fmaf(wb, C.y, DO[r].y);
                        }
                    } else {
                        D[r] = C;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                if constexpr (!PAR) {
                    const float2* tH = tH0 + (size_t)c * P.nH3span + H3lo + hbeg;
#pragma unroll
                    for (int h = 0; h < HC; ++h) {
                        if (h < hmin || h < hcnt) {
                            const float t3 = t3base + (float)h * dt3;
                            float2 acc = D[N];
#pragma unroll
                            for (int r = N - 1; r >= 0; --r)
                                acc = make_float2(D[r].x - t3 * acc.y, D[r].y + t3 * acc.x);
                            const float2 e3 = tH[h];
                            F[h].x += e3.x * acc.x - e3.y * acc.y;
                            F[h].y += e3.x * acc.y + e3.y * acc.x;
                        }
                    }
                }
            }
        };
        if constexpr (PAR) {
            level_b(0, std::true_type{});
            for (int c = 1; c < P.nclass; ++c) level_b(c, std::false_type{});
        } else {
            for (int c = 0; c < P.nclass; ++c) level_b(c, std::false_type{});
        }
        if constexpr (MULTI) {
            if constexpr (PAR) {
#pragma unroll
                for (int h = 0; h < HC; ++h)
                    if (h < hmin || h < hcnt) I[h] += parity_eval<N>((h & 1) ? DO : DE, t3base + (float)h * dt3);
            } else {
#pragma unroll
                for (int h = 0; h < HC; ++h) I[h] += F[h].x * F[h].x + F[h].y * F[h].y;
            }
            __syncthreads();                 // every thread has read Bs before it is cleared
        }
    }
    const int i3b = k3 + n3 * (H3lo + hbeg) - P.g0[2];       // output index of h = 0
    const RowOut ro = row_out(P, w, i2, i3b);
    const bool full = __ballot(active) == ~0ull;
    auto val = [&](int h) -> float {
        if constexpr (MULTI) return I[h];
        else if constexpr (PAR) return parity_eval<N>((h & 1) ? DO : DE, t3base + (float)h * dt3);
        else return F[h].x * F[h].x + F[h].y * F[h].y;
    };
    if (w.mirror) write_row<HC, true>(ro, full, active, hmin, hcnt, 1.f, val);
    else write_row<HC, false>(ro, full, active, hmin, hcnt, 1.f, val);
}

template <int N, int HC, bool MULTI, bool PAR>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu((!MULTI && PAR) ? 6 : 4)))
void k_recombine_folded(RecombParams P) { recombine_folded_body<N, HC, MULTI, PAR, RecombParams>(P, blockIdx.x); }
template <int N, int HC, bool MULTI, bool PAR>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu((!MULTI && PAR) ? 6 : 4)))
void k_recombine_folded_merged(const RecombParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) recombine_folded_body<N, HC, MULTI, PAR, const RecombParams&>(tab[d], bx);
}

// ---------------------------------------------------------------------------- nuclear launchers
// The nuclear and folded forms are instantiated per Taylor order in the recombine_o*.hip
// units (explicit instantiations of launch_nuc_hc / launch_nuc_hi), which include this file
// with DSX_RECOMBINE_PART defined and compile in parallel; this unit declares them extern.
template <typename K>
static hipError_t set_lds(K kernel, size_t lds)
{
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int N, int HC, bool MULTI, bool PAR>
static hipError_t launch_nuc_v(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    hipError_t e = set_lds(k_recombine_nuclear<N, HC, MULTI, PAR>, lds);
    if (e != hipSuccess) return e;
    return dispatch(k_recombine_nuclear<N, HC, MULTI, PAR>, k_recombine_nuclear_merged<N, HC, MULTI, PAR>, p.nwork,
                    block, lds, st, p);
}

template <int N, int HC, bool MULTI, bool PAR>
static hipError_t launch_fold_v(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    hipError_t e = set_lds(k_recombine_folded<N, HC, MULTI, PAR>, lds);
    if (e != hipSuccess) return e;
    return dispatch(k_recombine_folded<N, HC, MULTI, PAR>, k_recombine_folded_merged<N, HC, MULTI, PAR>, p.nwork,
                    block, lds, st, p);
}

template <int N, int HC>
static hipError_t launch_nuc(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    const bool multi = p.M > 1 || p.variant == 1;
    const bool par = p.parity != 0 && p.variant != 2;
    if (p.fold) {
        if (multi) return par ? launch_fold_v<N, HC, true, true>(p, block, lds, st)
                              : launch_fold_v<N, HC, true, false>(p, block, lds, st);
        return par ? launch_fold_v<N, HC, false, true>(p, block, lds, st)
                   : launch_fold_v<N, HC, false, false>(p, block, lds, st);
    }
    if (multi) return par ? launch_nuc_v<N, HC, true, true>(p, block, lds, st)
                          : launch_nuc_v<N, HC, true, false>(p, block, lds, st);
    return par ? launch_nuc_v<N, HC, false, true>(p, block, lds, st)
               : launch_nuc_v<N, HC, false, false>(p, block, lds, st);
}

template <int N>
hipError_t launch_nuc_hc(const RecombParams& p, int hc, int block, size_t lds, hipStream_t st)
{
    switch (hc) {
        case 4: return launch_nuc<N, 4>(p, block, lds, st);
        case 8: return launch_nuc<N, 8>(p, block, lds, st);
        case 17: return launch_nuc<N, 17>(p, block, lds, st);
        case 32: return launch_nuc<N, 32>(p, block, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// Orders above kMaxOrderFast: the class form (no folding, no parity sets), H3 runs of 4 or 8.
template <int N>
hipError_t launch_nuc_hi(const RecombParams& p, int hc, int block, size_t lds, hipStream_t st)
{
    if (p.fold || p.parity) return hipErrorInvalidValue;
    const bool multi = p.M > 1 || p.variant == 1;
    switch (hc) {
        case 4: return multi ? launch_nuc_v<N, 4, true, false>(p, block, lds, st)
                             : launch_nuc_v<N, 4, false, false>(p, block, lds, st);
        case 8: return multi ? launch_nuc_v<N, 8, true, false>(p, block, lds, st)
                             : launch_nuc_v<N, 8, false, false>(p, block, lds, st);
        default: return hipErrorInvalidValue;
    }
}

#ifndef DSX_RECOMBINE_PART

// ---------------------------------------------------------------------------- magnetic
// the form factor f_mag of Eq. mag_sf
__device__ __forceinline__ float mag_ff(const float* f, float s2) { return site_ff(f, s2); }

// Debye-Waller factor T_mu(G) of Sec. III.A, Eq. dw, in its order-N Taylor form,
//   T_mu(G) = sum_{p+q+r<=N} (i t1)^p/p! (i t2)^q/q! (i t3)^r/r! <u1^p u2^q u3^r>_mu,
// t_a = 2 pi g_a, <.> the mean over the site's occupied atoms and the configurations
// (dwc), sum-factorised like the nuclear recombination: p per block (this function, in
// float64, into LDS A[mu][pair (q, r)]), q per thread (dw_level_b), r per voxel (Horner).
__device__ void dw_level_a(const RecombParams& P, double tau1, float2* A)
{
    const int N = P.dw_order, QR = n_pairs(N);
    for (int idx = threadIdx.x; idx < P.S * QR; idx += blockDim.x) {
        const int mu = idx / QR, j = idx - mu * QR;
        int e = 0;
        while ((e + 1) * (e + 2) / 2 <= j) ++e;
        const int r = j - e * (e + 1) / 2, q = e - r;
        const double* c = P.dwc + (size_t)mu * P.dwT;
        double ar = 0.0, ai = 0.0, mag = 1.0;     // (i t1)^p / p! = i^p mag
        for (int p = 0; p + e <= N; ++p) {
            const double v = mag * c[mono_index(p, q, r)];
            switch (p & 3) {
                case 0: ar += v; break;
                case 1: ai += v; break;
                case 2: ar -= v; break;
                default: ai -= v; break;
            }
            mag *= tau1 / (p + 1);
        }
        A[idx] = make_float2((float)ar, (float)ai);
    }
}

// B[r] = sum_q (i t2)^q/q! A[(q, r)] / r! for one site (the 1/r! folded in here).
__device__ __forceinline__ void dw_level_b(const float2* A, int N, float tau2, float2 (&B)[kMaxOrder + 1])
{
#pragma unroll
    for (int r = 0; r <= kMaxOrder; ++r) {
        B[r] = make_float2(0.f, 0.f);
        if (r > N) continue;
        float mag = 1.f, rf = 1.f;
        for (int k = 2; k <= r; ++k) rf *= (float)k;
        for (int q = 0; q + r <= N; ++q) {
            const float2 a = A[pair_index(q, r)];
            float2 v = make_float2(a.x * mag, a.y * mag);
            if (q & 1) v = make_float2(-v.y, v.x);          // times i
            if (q & 2) v = make_float2(-v.x, -v.y);         // times -1
            B[r].x += v.x; B[r].y += v.y;
            mag *= tau2 / (float)(q + 1);
        }
        B[r].x /= rf; B[r].y /= rf;
    }
}

// sum_r (i t3)^r B[r] (Horner).
__device__ __forceinline__ float2 dw_level_c(const float2 (&B)[kMaxOrder + 1], int N, float tau3)
{
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int r = kMaxOrder; r >= 0; --r) {
        if (r > N) continue;
        acc = make_float2(B[r].x - tau3 * acc.y, B[r].y + tau3 * acc.x);
    }
    return acc;
}

// DW: the sites carry Debye-Waller factors T_mu(G) (Eq. dw); each site is then taken
// on its own at level C instead of summed into its class first.
template <int HC, bool DW, class PT>
__device__ __forceinline__ void recombine_magnetic_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    BlockWork w;
    if (!decode_block(P, w, bx)) return;
    float2* Bs = smem;                    // [sites of the chunk][3][n3]
    float2* Xs = smem + P.bs_elems;       // [2][sites of the chunk][3][nh] staging
    float2* tHs = Xs + P.xs_elems;        // [nclass][nH3span]
    float2* dwA = tHs + P.nclass * P.nH3span;   // DW: [S][pairs]
    const float2* tH0 = stage_class_phases(P, tHs);
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3, nh = P.nh;
    const int SFnh = P.SF * nh;
    const int nitems = (w.h2b - w.h2a) * n3 * P.nchunk3;
    const int item = threadIdx.x;
    const bool active = item < nitems;
    int k3 = 0, ch = 0, h2 = w.h2a;
    if (active) {
        k3 = item % n3;
        const int r = item / n3;
        ch = r % P.nchunk3;
        h2 = w.h2a + r / P.nchunk3;
    }
    const int G2 = w.k2 + n2 * (w.H2lo + h2);
    const int i2 = G2 - P.g0[1];
    int H3lo, nH3;
    hrange(k3, n3, P.g0[2], P.cnt[2], H3lo, nH3);
    const int hbeg = ch * HC;
    const int hcnt = active ? max(0, min(HC, nH3 - hbeg)) : 0;
    // Cartesian Q = g1 a* + g2 b* + g3 c*
    const float g1 = (float)((double)w.G1 / (double)n1);
    const float g2 = (float)((double)G2 / (double)n2);
    const float q12x = g1 * P.recip[0] + g2 * P.recip[3];
    const float q12y = g1 * P.recip[1] + g2 * P.recip[4];
    const float q12z = g1 * P.recip[2] + g2 * P.recip[5];
    const float inv16pi2 = 1.f / (16.f * 9.8696044010893586f);
    const int Ndw = DW ? P.dw_order : 0;
    const float tau2 = (float)(6.283185307179586 * (double)G2 / (double)n2);
    if constexpr (DW) dw_level_a(P, 6.283185307179586 * (double)w.G1 / (double)n1, dwA);

    float I[HC];
#pragma unroll
    for (int h = 0; h < HC; ++h) I[h] = 0.f;
    const size_t col = ((size_t)w.k1 * n2 + w.k2) * SFnh;
    const size_t colm = ((size_t)((n1 - w.k1) % n1) * n2 + (n2 - w.k2) % n2) * SFnh;

    for (int m = 0; m < P.M; ++m) {
        float2 F[HC][3];
#pragma unroll
        for (int h = 0; h < HC; ++h)
#pragma unroll
            for (int c = 0; c < 3; ++c) F[h][c] = make_float2(0.f, 0.f);
        const float2* Xm = P.X + (size_t)m * n1 * n2 * SFnh;
        for (int sc = 0; sc < P.nsc; ++sc) {
            const int s0 = P.sc_start[sc], s1 = P.sc_start[sc + 1];
            const int ns = s1 - s0;
            // level A: stage the chunk's spin spectra of column (k1, k2) and of the
            // mirrored column, then apply b_mu e^{2 pi i g1 r_mu1}
            __syncthreads();
            for (int sl = 0; sl < ns; ++sl) {
                const int mu = P.site_of[s0 + sl];
                stage_copy(Xs + sl * 3 * nh, Xm + col + (size_t)mu * 3 * nh, 3 * nh);
                stage_copy(Xs + (ns + sl) * 3 * nh, Xm + colm + (size_t)mu * 3 * nh, 3 * nh);
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < ns * 3 * n3; idx += blockDim.x) {
                const int kk = idx % n3;
                const int rj = idx / n3;
                const int comp = rj % 3;
                const int sl = rj / 3;
                const int mu = P.site_of[s0 + sl];
                float2 x;
                if (kk < nh) x = Xs[(sl * 3 + comp) * nh + kk];
                else { x = Xs[ns * 3 * nh + (sl * 3 + comp) * nh + (n3 - kk)]; x.y = -x.y; }
                Bs[idx] = cmulf(P.tab1[(size_t)mu * P.cnt[0] + w.i1], x);
            }
            __syncthreads();
            if (hcnt > 0) {
                int sp = s0;
                while (sp < s1) {
                    const int c = P.class_of[sp];
                    // a class at once, or (DW) one site at a time
                    int se = sp + 1;
                    while (!DW && se < s1 && P.class_of[se] == c) ++se;
                    float2 D[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                    for (int sl = sp - s0; sl < se - s0; ++sl) {
                        const int mu = P.site_of[s0 + sl];
                        const float2 ph = cmulf(P.tab2[(size_t)mu * P.cnt[1] + i2],
                                                P.tabK3[(size_t)mu * n3 + k3]);
                        const float2* Bp = Bs + (size_t)sl * 3 * n3 + k3;
#pragma unroll
                        for (int comp = 0; comp < 3; ++comp) {
                            const float2 v = cmulf(ph, Bp[comp * n3]);
                            D[comp].x += v.x;
                            D[comp].y += v.y;
                        }
                    }
                    float2 Bdw[kMaxOrder + 1];
                    if constexpr (DW) dw_level_b(dwA + (size_t)P.site_of[sp] * n_pairs(Ndw), Ndw, tau2, Bdw);
                    const float2* tH = tH0 + (size_t)c * P.nH3span;
                    const float* ffc = P.ff[sp];
#pragma unroll
                    for (int h = 0; h < HC; ++h) {
                        if (h < hcnt) {
                            const int H3 = H3lo + hbeg + h;
                            float2 e3 = tH[H3];
                            if (!P.ff_uniform) {
                                const float g3 = (float)(k3 + n3 * H3) / (float)n3;
                                const float qx = q12x + g3 * P.recip[6], qy = q12y + g3 * P.recip[7],
                                            qz = q12z + g3 * P.recip[8];
                                const float f = mag_ff(ffc, (qx * qx + qy * qy + qz * qz) * inv16pi2);
                                e3.x *= f; e3.y *= f;
                            }
                            if constexpr (DW) {
                                const float tau3 = 6.283185307f * ((float)(k3 + n3 * H3) / (float)n3);
                                e3 = cmulf(e3, dw_level_c(Bdw, Ndw, tau3));
                            }
#pragma unroll
                            for (int comp = 0; comp < 3; ++comp) {
                                F[h][comp].x += e3.x * D[comp].x - e3.y * D[comp].y;
                                F[h][comp].y += e3.x * D[comp].y + e3.y * D[comp].x;
                            }
                        }
                    }
                    sp = se;
                }
            }
        }
        // perpendicular projection and |F_perp|^2
#pragma unroll
        for (int h = 0; h < HC; ++h) {
            if (h < hcnt) {
                const int H3 = H3lo + hbeg + h;
                const float g3 = (float)(k3 + n3 * H3) / (float)n3;
                const float qx = q12x + g3 * P.recip[6], qy = q12y + g3 * P.recip[7],
                            qz = q12z + g3 * P.recip[8];
                const float q2 = qx * qx + qy * qy + qz * qz;
                if (q2 > 0.f) {
                    const float iq = rsqrtf(q2);
                    const float ex = qx * iq, ey = qy * iq, ez = qz * iq;
                    const float px = ex * F[h][0].x + ey * F[h][1].x + ez * F[h][2].x;
                    const float py = ex * F[h][0].y + ey * F[h][1].y + ez * F[h][2].y;
                    float v = 0.f;
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp)
                        v += F[h][comp].x * F[h][comp].x + F[h][comp].y * F[h][comp].y;
                    v -= px * px + py * py;
                    if (P.ff_uniform) {
                        const float f = mag_ff(P.ff[0], q2 * inv16pi2);
                        v *= f * f;
                    }
                    I[h] += v;
                }
            }
        }
    }
    if (hcnt > 0) {
        float* orow = P.out + P.ooff + ((size_t)w.i1 * P.cnt[1] + i2) * P.opitch;
        float* mrow = P.out + P.ooff + ((size_t)(P.cnt[0] - 1 - w.i1) * P.cnt[1] + (P.cnt[1] - 1 - i2)) * P.opitch;
#pragma unroll
        for (int h = 0; h < HC; ++h) {
            if (h < hcnt) {
                const int i3 = k3 + n3 * (H3lo + hbeg + h) - P.g0[2];
                const float v = I[h] * P.scale;
                orow[i3] = v;
                if (w.mirror) mrow[P.cnt[2] - 1 - i3] = v;
            }
        }
    }
}

template <int HC, bool DW>
__global__ __launch_bounds__(512) void k_recombine_magnetic(RecombParams P) { recombine_magnetic_body<HC, DW, RecombParams>(P, blockIdx.x); }
template <int HC, bool DW>
__global__ __launch_bounds__(512) void k_recombine_magnetic_merged(const RecombParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) recombine_magnetic_body<HC, DW, const RecombParams&>(tab[d], bx);
}

int recombine_max_threads(int hc, int magnetic)
{
    (void)hc; (void)magnetic;
    return 512;
}


// Row-staged form of the magnetic recombination (sites without a Debye-Waller factor).
// A block takes rows h2a..h2b of column (k1, k2) in plane G1 (and, with one configuration
// and every r_mu1 a multiple of 1/q1, in up to three more planes G1 + p q1 n1, whose site
// phases e^{2 pi i g1 r_mu1} are plane G1's, so levels A and B serve all of them); its
// threads cover the box's G3 (one output column each, so a row is written by consecutive
// threads):
//   level A  Bs[site][comp][k3] = b_mu e^{2 pi i (g1 r_mu1 + k3 r_mu3 / n3)} M_comp(k1, k2, k3),
//            one site chunk at a time, read straight from the spin spectra of the column
//            (k3 <= n3/2) and of its mirror (the rest, through X(k) = conj X(-k));
//   level B  D[row][class][comp][k3] += sum over the chunk's sites of the class of
//            e^{2 pi i g2 r_mu2} Bs (when every r_mu2 is a multiple of 1/q2, rows whose
//            H2 agree mod q2 have equal phases: the first q2 rows stand for all of
//            them); then, when every r_c3 of the classes is a multiple
//            of 1/q and the form factor is the same for every site, the classes are
//            summed per residue of H3 mod q, in place (q <= nclass):
//            E[row][j][comp][k3] = sum_c e^{2 pi i H3_j r_c3} D  (H3_j = j mod q);
//   level C  per voxel of the thread's column: F_comp = E[row][H3 mod q][comp][k3], or
//            sum_c e^{2 pi i H3 r_c3} f_c(|Q|) D, then F_perp = F - Qhat (Qhat . F),
//            |F_perp|^2 and f(|Q|)^2 (Eqs. mag_sf, mag_projection).  One configuration:
//            each value is stored as it is made; several: accumulated in registers.
// The form factor uses the hardware exponential (relative error ~1e-6 at the arguments
// a s^2 <= 30 met here).
__device__ __forceinline__ float mag_ff_fast(const float* f, float s2) {
    return f[0] * __expf(-f[1] * s2) + f[2] * __expf(-f[3] * s2) + f[4] * __expf(-f[5] * s2) + f[6];
}

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
}

// NCT: the number of r3 classes when the classes are summed per residue of H3 mod q
// (then at most kMagRowsMaxClasses, and the residue sums unroll over it), else 0.
template <bool MULTI, int NCT, class PT>
__device__ __forceinline__ void recombine_magnetic_rows_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    __shared__ int cls[kMaxSites + 1];
    __shared__ float2 t1s[kMaxSites];
    __shared__ float2 phq[NCT > 0 ? NCT * NCT : 1];   // [j][c]: e^{2 pi i H3_j r_c3}, H3_j of residue j
    __shared__ float4 ffrow[kMagRowsMaxRows];         // separable form factor: the rows' g2 parts
    BlockWork w;
    if (!decode_block(P, w, bx)) return;
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3, nh = P.nh, S = P.S, NC = P.nclass, q = P.qmod;
    const int rows = w.h2b - w.h2a, cnt3 = P.cnt[2], q2 = P.qmod2;
    // staged rows: with every r_mu2 a multiple of 1/q2, row r has the site phases of row
    // r mod q2 (their H2 differ by a multiple of q2), so only the first q2 are staged
    const int rowsB = q2 > 0 ? min(rows, q2) : rows;
    float2* D = smem;                              // [rowsB][NC][3][n3]; then E [rowsB][q][3][n3]
    float2* tK3 = D + rowsB * NC * 3 * n3;         // [S][n3]   (sorted positions)
    float2* t2 = tK3 + S * n3;                     // [rowsB][S]
    float2* tHs = t2 + rowsB * S;                  // [NC][nH3span]
    float2* Bs = tHs + NC * P.nH3span;             // [csites][3][n3]
    const float2* tH0 = stage_class_phases(P, tHs);
    const float rn3 = 1.f / (float)n3, rS = 1.f / (float)S, rNC = 1.f / (float)NC;
    for (int idx = threadIdx.x; idx < S * n3; idx += blockDim.x) {
        const int i = qdiv_r(idx, n3, rn3), k = idx - i * n3;
        tK3[idx] = P.tabK3[(size_t)P.site_of[i] * n3 + k];
    }
    for (int idx = threadIdx.x; idx < rowsB * S; idx += blockDim.x) {
        const int r = qdiv_r(idx, S, rS), i = idx - r * S;
        const int i2 = w.k2 + n2 * (w.H2lo + w.h2a + r) - P.g0[1];
        t2[idx] = P.tab2[(size_t)P.site_of[i] * P.cnt[1] + i2];
    }
    for (int i = threadIdx.x; i <= NC; i += blockDim.x) cls[i] = P.class_start[i];
    for (int i = threadIdx.x; i < S; i += blockDim.x) t1s[i] = P.tab1[(size_t)P.site_of[i] * P.cnt[0] + w.i1];
    const int SFnh = P.SF * nh;
    const size_t col = ((size_t)w.k1 * n2 + w.k2) * SFnh;
    const size_t colm = ((size_t)((n1 - w.k1) % n1) * n2 + (n2 - w.k2) % n2) * SFnh;
    // the thread's output column i3 (the launch has at least cnt3 threads)
    const int i3 = threadIdx.x;
    const bool active = i3 < cnt3;
    const int G3 = P.g0[2] + i3;
    const int H3 = floordiv(G3, n3);
    const int k3 = G3 - n3 * H3;
    const int jq = q > 0 ? H3 - q * floordiv(H3, q) : 0;
    const int ebase = jq * 3 * n3 + k3;            // the thread's residue sums within a staged row
    const int erow = NC * 3 * n3;                  // float2 per staged row
    const float inv16pi2 = 1.f / (16.f * 9.8696044010893586f);
    const float g3 = (float)((double)G3 / (double)n3);
    const float rn2f = (float)(1.0 / (double)n2);
    // the block's G1 planes (H1 agreeing mod qmod1: their site phases are plane 0's)
    const int wbits = P.work[bx].w;
    const int npl = 1 + ((wbits >> 28) & 3);
    // a separable form factor: e^{-a s^2} = e^{-a |q13|^2 / 16 pi^2} e^{-a g2^2 |b*|^2 / 16 pi^2}
    // (b* orthogonal to a* and c*), the first factor per thread and plane, the second per row
    const bool sep = P.ff_uniform && P.ff_sep;
    if (sep) {
        const float* f = P.ff[0];
        const float b2sq = P.recip[3] * P.recip[3] + P.recip[4] * P.recip[4] + P.recip[5] * P.recip[5];
        for (int r = threadIdx.x; r < rows; r += blockDim.x) {
            const float g2 = (float)(w.k2 + n2 * (w.H2lo + w.h2a + r)) * rn2f;
            const float t = g2 * g2 * b2sq * inv16pi2;
            ffrow[r] = make_float4(__expf(-f[1] * t), __expf(-f[3] * t), __expf(-f[5] * t), 0.f);
        }
    }
    const size_t plane = (size_t)P.cnt[1] * P.opitch;
    float I[MULTI ? kMagRowsMaxRows : 1];
#pragma unroll
    for (int r = 0; r < (MULTI ? kMagRowsMaxRows : 1); ++r) I[r] = 0.f;

    for (int m = 0; m < P.M; ++m) {
        const float2* Xm = P.X + (size_t)m * n1 * n2 * SFnh;
        __syncthreads();
        for (int idx = threadIdx.x; idx < rowsB * NC * 3 * n3; idx += blockDim.x) D[idx] = make_float2(0.f, 0.f);
        for (int s0 = 0; s0 < S; s0 += P.csites) {
            const int ns = min(P.csites, S - s0);
            __syncthreads();
            // level A (with the k3 phase of the site)
            for (int idx = threadIdx.x; idx < ns * 3 * n3; idx += blockDim.x) {
                const int rj = qdiv_r(idx, n3, rn3);
                const int kk = idx - rj * n3;
                const int sl = rj / 3, comp = rj - 3 * sl;
                const size_t f = ((size_t)P.site_of[s0 + sl] * 3 + comp) * nh;
                float2 x;
                if (kk < nh) x = Xm[col + f + kk];
                else { x = Xm[colm + f + (n3 - kk)]; x.y = -x.y; }
                Bs[idx] = cmulf(cmulf(t1s[s0 + sl], tK3[(s0 + sl) * n3 + kk]), x);
            }
            __syncthreads();
            // level B: one (row, class, k3) per thread, the chunk's sites of the class
            for (int idx = threadIdx.x; idx < rowsB * NC * n3; idx += blockDim.x) {
                const int rc = qdiv_r(idx, n3, rn3);
                const int kk = idx - rc * n3;
                const int r = qdiv_r(rc, NC, rNC);
                const int c = rc - r * NC;
                const int i0 = max(cls[c], s0), i1 = min(cls[c + 1], s0 + ns);
                if (i0 >= i1) continue;
                float2 acc[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                for (int i = i0; i < i1; ++i) {
                    const float2 ph = t2[r * S + i];
                    const float2* b = Bs + (size_t)(i - s0) * 3 * n3 + kk;
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) cmac(acc[comp], ph, b[comp * n3]);
                }
                float2* d = D + (size_t)rc * 3 * n3 + kk;
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) {
                    d[comp * n3].x += acc[comp].x;
                    d[comp * n3].y += acc[comp].y;
                }
            }
        }
        __syncthreads();
        // classes summed per residue of H3 mod q, in place: one (row, comp, k3) per
        // thread reads its NCT classes' D, then writes E over the first q of them (the
        // block's q x NCT phases staged once; a residue with no H3 in the box stays 0)
        if constexpr (NCT > 0) {
            if (m == 0) {
                for (int t = threadIdx.x; t < NCT * NCT; t += blockDim.x) {
                    const int j = t / NCT, c = t - j * NCT;
                    const int h = P.H3min + ((j - P.H3min) % q + q) % q;   // an H3 of residue j
                    phq[t] = (j < q && h - P.H3min < P.nH3span) ? tH0[c * P.nH3span + h] : make_float2(0.f, 0.f);
                }
                __syncthreads();
            }
            for (int idx = threadIdx.x; idx < rowsB * 3 * n3; idx += blockDim.x) {
                const int rc = qdiv_r(idx, n3, rn3);
                const int kk = idx - rc * n3;
                const int r = rc / 3, comp = rc - 3 * r;
                float2* d = D + (size_t)r * NCT * 3 * n3 + comp * n3 + kk;
                float2 dv[NCT];
#pragma unroll
                for (int c = 0; c < NCT; ++c) dv[c] = d[c * 3 * n3];
#pragma unroll
                for (int j = 0; j < NCT; ++j) {
                    if (j < q) {
                        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
                        for (int c = 0; c < NCT; ++c) cmac(acc, phq[j * NCT + c], dv[c]);
                        d[j * 3 * n3] = acc;
                    }
                }
            }
            __syncthreads();
        }
        // level C: the thread's column, every row of every plane of the block
        for (int pl = 0; pl < npl && active; ++pl) {
            const int G1 = w.G1 + pl * P.qmod1 * n1;
            const int i1 = G1 - P.g0[0];
            const bool mirror = (wbits >> (24 + pl)) & 1;
            const float g1 = (float)((double)G1 / (double)n1);
            const float q13x = g1 * P.recip[0] + g3 * P.recip[6];
            const float q13y = g1 * P.recip[1] + g3 * P.recip[7];
            const float q13z = g1 * P.recip[2] + g3 * P.recip[8];
            float e13a = 0.f, e13b = 0.f, e13c = 0.f;
            if (sep) {
                const float* f = P.ff[0];
                const float s13 = (q13x * q13x + q13y * q13y + q13z * q13z) * inv16pi2;
                e13a = f[0] * __expf(-f[1] * s13);
                e13b = f[2] * __expf(-f[3] * s13);
                e13c = f[4] * __expf(-f[5] * s13);
            }
            float* const orow0 = P.out + P.ooff + (size_t)i1 * plane + i3;
            float* const mrow0 = P.out + P.ooff + (size_t)(P.cnt[0] - 1 - i1) * plane + (P.cnt[2] - 1 - i3);
            int rd = 0;                            // the staged row holding row r's sums
            for (int r = 0; r < rows; ++r, rd = (rd + 1 == rowsB) ? 0 : rd + 1) {
                const int G2 = w.k2 + n2 * (w.H2lo + w.h2a + r);
                const float g2 = (float)G2 * rn2f;
                const float qx = q13x + g2 * P.recip[3];
                const float qy = q13y + g2 * P.recip[4];
                const float qz = q13z + g2 * P.recip[5];
                const float q2 = qx * qx + qy * qy + qz * qz;
                const float s2 = q2 * inv16pi2;
                float2 F[3];
                if (NCT > 0) {
                    const float2* e = D + rd * erow + ebase;
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) F[comp] = e[comp * n3];
                } else {
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) F[comp] = make_float2(0.f, 0.f);
                    const float2* d = D + (size_t)rd * NC * 3 * n3 + k3;
                    const float2* th = tH0 + H3;
                    for (int c = 0; c < NC; ++c) {
                        float2 e3 = th[c * P.nH3span];
                        if (!P.ff_uniform) {
                            const float f = mag_ff_fast(P.ff[cls[c]], s2);
                            e3.x *= f; e3.y *= f;
                        }
#pragma unroll
                        for (int comp = 0; comp < 3; ++comp) cmac(F[comp], e3, d[(c * 3 + comp) * n3]);
                    }
                }
                // |F_perp|^2 = |F|^2 - |Q.F|^2 / |Q|^2 (0 at Q = 0), times f(|Q|)^2
                const float pr = qx * F[0].x + qy * F[1].x + qz * F[2].x;
                const float pim = qx * F[0].y + qy * F[1].y + qz * F[2].y;
                float f2 = 0.f;
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) f2 += F[comp].x * F[comp].x + F[comp].y * F[comp].y;
                float val = fmaf(-(pr * pr + pim * pim), __builtin_amdgcn_rcpf(q2), f2);
                if (sep) {
                    const float4 e2 = ffrow[r];
                    const float f = fmaf(e13a, e2.x, fmaf(e13b, e2.y, fmaf(e13c, e2.z, P.ff[0][6])));
                    val *= f * f;
                } else if (P.ff_uniform) {
                    const float f = mag_ff_fast(P.ff[0], s2);
                    val *= f * f;
                }
                val = q2 > 0.f ? val : 0.f;
                if constexpr (MULTI) {
#pragma unroll
                    for (int rr = 0; rr < kMagRowsMaxRows; ++rr)
                        if (rr == r) I[rr] += val;
                } else {
                    const int i2 = G2 - P.g0[1];
                    const float o = val * P.scale;
                    orow0[(size_t)i2 * P.opitch] = o;
                    if (mirror) mrow0[(size_t)(P.cnt[1] - 1 - i2) * P.opitch] = o;
                }
            }
        }
    }
    if constexpr (MULTI) {
        // several configurations: one plane per block (the planner groups no planes)
        float* const orow0 = P.out + P.ooff + (size_t)w.i1 * plane + i3;
        float* const mrow0 = P.out + P.ooff + (size_t)(P.cnt[0] - 1 - w.i1) * plane + (P.cnt[2] - 1 - i3);
        if (active) {
#pragma unroll
            for (int r = 0; r < kMagRowsMaxRows; ++r) {
                if (r < rows) {
                    const int i2 = w.k2 + n2 * (w.H2lo + w.h2a + r) - P.g0[1];
                    const float o = I[r] * P.scale;
                    orow0[(size_t)i2 * P.opitch] = o;
                    if (w.mirror) mrow0[(size_t)(P.cnt[1] - 1 - i2) * P.opitch] = o;
                }
            }
        }
    }
}

template <bool MULTI, int NCT>
__global__ __launch_bounds__(kMagRowsMaxThreads) void k_recombine_magnetic_rows(RecombParams P) { recombine_magnetic_rows_body<MULTI, NCT, RecombParams>(P, blockIdx.x); }
template <bool MULTI, int NCT>
__global__ __launch_bounds__(kMagRowsMaxThreads) void k_recombine_magnetic_rows_merged(const RecombParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) recombine_magnetic_rows_body<MULTI, NCT, const RecombParams&>(tab[d], bx);
}

template <bool MULTI, int NCT>
static hipError_t launch_mag_rows_v(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    hipError_t e = set_lds(k_recombine_magnetic_rows<MULTI, NCT>, lds);
    if (e != hipSuccess) return e;
    return dispatch(k_recombine_magnetic_rows<MULTI, NCT>, k_recombine_magnetic_rows_merged<MULTI, NCT>, p.nwork, block,
                    lds, st, p);
}

template <bool MULTI>
static hipError_t launch_mag_rows(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    // residue sums for up to four classes (the unrolled sums keep the block's q x NC
    // phases in registers); more classes, or no residue grid, take level C per class,
    // which is exact for any q
    if (p.qmod <= 0 || p.nclass > 4) return launch_mag_rows_v<MULTI, 0>(p, block, lds, st);
    switch (p.nclass) {
        case 1: return launch_mag_rows_v<MULTI, 1>(p, block, lds, st);
        case 2: return launch_mag_rows_v<MULTI, 2>(p, block, lds, st);
        case 3: return launch_mag_rows_v<MULTI, 3>(p, block, lds, st);
        default: return launch_mag_rows_v<MULTI, 4>(p, block, lds, st);
    }
}

hipError_t launch_recombine_magnetic_rows(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    if (p.nwork <= 0) return hipSuccess;
    if (block < p.cnt[2] || block > kMagRowsMaxThreads || p.rows > kMagRowsMaxRows) return hipErrorInvalidValue;
    if (p.qmod > 0 && (p.qmod > p.nclass || p.nclass > kMagRowsMaxClasses)) return hipErrorInvalidValue;
    if (p.M > 1 && p.qmod1 > 0) return hipErrorInvalidValue;   // grouped planes: one configuration
    return p.M > 1 ? launch_mag_rows<true>(p, block, lds, st) : launch_mag_rows<false>(p, block, lds, st);
}

// ---------------------------------------------------------------------------- direct form
// Taylor order 0 (occupancies only, one field per site): every voxel is computed on its
// own, F_m(G) = sum_mu b_mu e^{2 pi i g.r_mu} X_mu,m(k), I(G) = scale sum_m |F_m(G)|^2.
// A wave takes 64 consecutive columns i3 of the box, one a lane, over kDirectRows
// consecutive rows (i1, i2): a lane's column fixes k3, H3 and the half of the spectra it
// reads, a row fixes k1, k2 and the spectra column for the whole wave (scalar registers,
// stepped from row to row), so a voxel costs its loads, |F|^2 and one store, and every
// load and store of a wave is one contiguous run.  For one or two sites x configurations
// this beats the levelled forms, whose blocks serve one column of the grid each.
constexpr int kDirectThreads = 256, kDirectRows = 16, kDirectGroup = 16;
constexpr int kDirectWaves = kDirectThreads / 64;

// a / b for a < 2^32 through the float64 reciprocal rb of b (relative error well below
// 2^-40): the estimate is within one of the quotient, and one remainder check makes it exact
__device__ __forceinline__ uint32_t udiv_exact(uint32_t a, uint32_t b, double rb)
{
    uint32_t q = (uint32_t)((double)a * rb);
    const long long r = (long long)a - (long long)q * b;
    q += (r >= (long long)b) ? 1u : 0u;
    q -= (r < 0) ? 1u : 0u;
    return q;
}
// 1/b in float64: the hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double rcp_refined(uint32_t b)
{
    const double d = (double)b;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}
// floor(a / b) for |a| < 2^22, b > 0, through the float reciprocal rb of b (a few ulp at
// most: the estimate is within one, then one remainder check)
__device__ __forceinline__ int floordiv_exact(int a, int b, float rb)
{
    int q = (int)floorf((float)a * rb);
    const int r = a - q * b;
    q += (r >= b) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

template <class PT>
__device__ __forceinline__ void recombine_direct_body(PT P, const int bx)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const uint32_t c2 = (uint32_t)P.cnt[2], c1 = (uint32_t)P.cnt[1];
    const uint32_t rows = (uint32_t)P.planes * c1;
    const uint32_t ncc = (c2 + 63) / 64;                                 // column chunks per row group
    const uint32_t gw = (uint32_t)bx * kDirectWaves + wave;
    const uint32_t rg = __builtin_amdgcn_readfirstlane(udiv_exact(gw, ncc, rcp_refined(ncc)));
    const uint32_t r0 = rg * kDirectRows;
    if ((uint64_t)r0 >= rows) return;
    const int i3 = (int)(gw - rg * ncc) * 64 + lane;
    if (i3 >= (int)c2) return;
    const int nr = (int)min((uint32_t)kDirectRows, rows - r0);
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3, nh = P.nh;
    const size_t SFnh = (size_t)P.SF * nh;
    const size_t cstride = (size_t)n1 * n2 * SFnh;     // between configurations
    const size_t fstride = (size_t)P.F * nh;           // between sites
    // the lane's column: k3, H3 and the half of the spectra (k3 >= nh reads conj X(-k))
    const int G3 = P.g0[2] + i3;
    const int H3 = floordiv_exact(G3, n3, __builtin_amdgcn_rcpf((float)n3));
    const int k3 = G3 - n3 * H3, h = H3 - P.H3min;
    const bool half = k3 >= nh;
    const int koff = half ? n3 - k3 : k3;
    // the wave's first row: (i1, i2) and k1, k2
    int i1 = __builtin_amdgcn_readfirstlane(udiv_exact(r0, c1, rcp_refined(c1)));
    int i2 = (int)(r0 - (uint32_t)i1 * c1);
    int k1 = __builtin_amdgcn_readfirstlane(P.g0[0] + i1 - n1 * floordiv_exact(P.g0[0] + i1, n1, __builtin_amdgcn_rcpf((float)n1)));
    int k2 = __builtin_amdgcn_readfirstlane(P.g0[1] + i2 - n2 * floordiv_exact(P.g0[1] + i2, n2, __builtin_amdgcn_rcpf((float)n2)));
    const int k20 = __builtin_amdgcn_readfirstlane(P.g0[1] - n2 * floordiv_exact(P.g0[1], n2, __builtin_amdgcn_rcpf((float)n2)));
    auto* op = gptr(P.out) + P.ooff + (size_t)r0 * P.opitch + i3;
    const bool one = P.S == 1;
    const int mu0 = P.site_of[0];
    const float2 t0 = ldg2(P.tab1, (size_t)mu0 * P.cnt[0]);
    const float b2s = (t0.x * t0.x + t0.y * t0.y) * P.scale;
    const float cj = half ? -1.f : 1.f;
    if (one) {
        // one site: the phase has modulus b, so |F_m|^2 = b^2 |X_m(k)|^2 exactly.  Rows go
        // in groups: the group's spectra offsets first (a direct-form spectrum has fewer than
        // 2^32 elements), then all its loads of a configuration in flight at once
        const float2* __restrict__ X0 = P.X + (size_t)mu0 * fstride;
        for (int g = 0; g < nr; g += kDirectGroup) {
            uint32_t colr[kDirectGroup];
#pragma unroll
            for (int r = 0; r < kDirectGroup; ++r) {
                const uint32_t colp = (uint32_t)((k1 * n2 + k2) * SFnh);
                const uint32_t colm = (uint32_t)(((k1 ? n1 - k1 : 0) * n2 + (k2 ? n2 - k2 : 0)) * SFnh);
                colr[r] = (half ? colm : colp) + (uint32_t)koff;
                if (++i2 == (int)c1) {
                    i2 = 0;
                    k2 = k20;
                    k1 = (k1 + 1 == n1) ? 0 : k1 + 1;
                } else {
                    k2 = (k2 + 1 == n2) ? 0 : k2 + 1;
                }
            }
            const int ng = min(kDirectGroup, nr - g);
            float I[kDirectGroup];
#pragma unroll
            for (int r = 0; r < kDirectGroup; ++r) I[r] = 0.f;
            for (int m = 0; m < P.M; ++m) {
                const float2* __restrict__ Xm = X0 + (size_t)m * cstride;
                float2 xv[kDirectGroup];
#pragma unroll
                for (int r = 0; r < kDirectGroup; ++r) xv[r] = r < ng ? ldg2(Xm, colr[r]) : make_float2(0.f, 0.f);
#pragma unroll
                for (int r = 0; r < kDirectGroup; ++r) I[r] += xv[r].x * xv[r].x + xv[r].y * xv[r].y;
            }
#pragma unroll
            for (int r = 0; r < kDirectGroup; ++r)
                if (r < ng) op[(size_t)r * P.opitch] = I[r] * b2s;
            op += (size_t)kDirectGroup * P.opitch;
        }
        return;
    }
    for (int r = 0; r < nr; ++r) {
        const size_t colp = ((size_t)k1 * n2 + k2) * SFnh;                                   // X(k)
        const size_t colm = ((size_t)(k1 ? n1 - k1 : 0) * n2 + (k2 ? n2 - k2 : 0)) * SFnh;   // X(-k), conjugated
        const size_t col = (half ? colm : colp) + (size_t)koff;
        float I = 0.f;
        for (int m = 0; m < P.M; ++m) {
            const float2* Xm = P.X + (size_t)m * cstride + col;
            float2 F = make_float2(0.f, 0.f);
            for (int s = 0; s < P.S; ++s) {
                const int mu = P.site_of[s];
                const float2 ph = cmulf(cmulf(ldg2(P.tab1, (size_t)mu * P.cnt[0] + i1), ldg2(P.tab2, (size_t)mu * c1 + i2)),
                                        cmulf(ldg2(P.tabK3, (size_t)mu * n3 + k3),
                                              ldg2(P.tabH3, (size_t)P.class_of[s] * P.nH3span + h)));
                float2 x = ldg2(Xm, (size_t)mu * fstride);
                x.y *= cj;
                F.x += ph.x * x.x - ph.y * x.y;
                F.y += ph.x * x.y + ph.y * x.x;
            }
            I += F.x * F.x + F.y * F.y;
        }
        I *= P.scale;
        *op = I;
        op += P.opitch;
        // next row: i2 (and k2) step by one, wrapping into the next plane
        if (++i2 == (int)c1) {
            i2 = 0;
            ++i1;
            k2 = k20;
            k1 = (k1 + 1 == n1) ? 0 : k1 + 1;
        } else {
            k2 = (k2 + 1 == n2) ? 0 : k2 + 1;
        }
    }
}

__global__ __launch_bounds__(kDirectThreads) void k_recombine_direct(RecombParams P)
{
    recombine_direct_body<RecombParams>(P, blockIdx.x);
}
__global__ __launch_bounds__(kDirectThreads) void k_recombine_direct_merged(const RecombParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) recombine_direct_body<const RecombParams&>(tab[d], bx);
}

hipError_t launch_recombine_direct(const RecombParams& p, hipStream_t st)
{
    if (p.planes < 0 || p.planes > p.cnt[0]) return hipErrorInvalidValue;
    const unsigned long long rows = (unsigned long long)p.planes * p.cnt[1];
    if (rows == 0 || p.cnt[2] == 0) return hipSuccess;
    if (rows * (unsigned long long)p.cnt[2] >= (1ULL << 32)) return hipErrorInvalidValue;
    const unsigned long long waves = (rows + kDirectRows - 1) / kDirectRows * ((p.cnt[2] + 63) / 64);
    return dispatch(k_recombine_direct, k_recombine_direct_merged, (unsigned)((waves + kDirectWaves - 1) / kDirectWaves),
                    kDirectThreads, 0, st, p);
}

// instantiated in recombine_o*.hip
extern template hipError_t launch_nuc_hc<0>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<1>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<2>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<3>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<4>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<5>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<6>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<7>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hc<8>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<9>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<10>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<11>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<12>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<13>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<14>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<15>(const RecombParams&, int, int, size_t, hipStream_t);
extern template hipError_t launch_nuc_hi<16>(const RecombParams&, int, int, size_t, hipStream_t);

hipError_t launch_recombine_nuclear(const RecombParams& p, int order, int hc, int block,
                                    size_t lds, hipStream_t st)
{
    if (p.nwork <= 0) return hipSuccess;
    switch (order) {
        case 9: return launch_nuc_hi<9>(p, hc, block, lds, st);
        case 10: return launch_nuc_hi<10>(p, hc, block, lds, st);
        case 11: return launch_nuc_hi<11>(p, hc, block, lds, st);
        case 12: return launch_nuc_hi<12>(p, hc, block, lds, st);
        case 13: return launch_nuc_hi<13>(p, hc, block, lds, st);
        case 14: return launch_nuc_hi<14>(p, hc, block, lds, st);
        case 15: return launch_nuc_hi<15>(p, hc, block, lds, st);
        case 16: return launch_nuc_hi<16>(p, hc, block, lds, st);
        case 0: return launch_nuc_hc<0>(p, hc, block, lds, st);
        case 1: return launch_nuc_hc<1>(p, hc, block, lds, st);
        case 2: return launch_nuc_hc<2>(p, hc, block, lds, st);
        case 3: return launch_nuc_hc<3>(p, hc, block, lds, st);
        case 4: return launch_nuc_hc<4>(p, hc, block, lds, st);
        case 5: return launch_nuc_hc<5>(p, hc, block, lds, st);
        case 6: return launch_nuc_hc<6>(p, hc, block, lds, st);
        case 7: return launch_nuc_hc<7>(p, hc, block, lds, st);
        case 8: return launch_nuc_hc<8>(p, hc, block, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <int HC, bool DW>
static hipError_t launch_mag_v(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    hipError_t e = set_lds(k_recombine_magnetic<HC, DW>, lds);
    if (e != hipSuccess) return e;
    return dispatch(k_recombine_magnetic<HC, DW>, k_recombine_magnetic_merged<HC, DW>, p.nwork, block, lds, st, p);
}

template <int HC>
static hipError_t launch_mag(const RecombParams& p, int block, size_t lds, hipStream_t st)
{
    return (p.dwc && p.dw_order > 0) ? launch_mag_v<HC, true>(p, block, lds, st)
                                     : launch_mag_v<HC, false>(p, block, lds, st);
}

hipError_t launch_recombine_magnetic(const RecombParams& p, int hc, int block, size_t lds,
                                     hipStream_t st)
{
    if (p.nwork <= 0) return hipSuccess;
    switch (hc) {
        case 4: return launch_mag<4>(p, block, lds, st);
        case 8: return launch_mag<8>(p, block, lds, st);
        case 17: return launch_mag<17>(p, block, lds, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------- Bragg, float64
// One 64-lane wave per unit-cell Bragg point H.  Lanes first form, one site each, the
// site factor b_mu f_mu(H) e^{2 pi i H.r_mu}; then they stride over the (site,
// monomial) pairs of a configuration, each adding S^{pqr}_{m,mu} times the monomial's
// (2 pi i)^{p+q+r} H1^p H2^q H3^r / (p! q! r!) times the site factor, so the whole sum
// over sites and monomials is one wave reduction (fixed order) per configuration.
// Lane 0 keeps the ensemble moments and writes I(H); all of it in float64.
template <int N, class PT>
__device__ __forceinline__ void bragg_nuclear_body(PT P, const int bx)
{
    // every product and sum rounded on its own (no contraction into FMAs): the kernel and
    // its merged twin then compute the same bits, and the variance of one configuration
    // cancels to exactly 0
#pragma clang fp contract(off)
    constexpr int T = n_monomials(N);
    __shared__ double Ar[3][N + 1], Ai[3][N + 1];
    __shared__ double Wr[kMaxSites], Wi[kMaxSites];
    __shared__ int mono_s[T];
    const int total = P.nH[0] * P.nH[1] * P.nH[2];
    const int idx = bx;
    if (idx >= total) return;
    const int lane = threadIdx.x;
    const int j3 = idx % P.nH[2], j2 = (idx / P.nH[2]) % P.nH[1], j1 = idx / (P.nH[2] * P.nH[1]);
    const int H[3] = {P.Hlo[0] + j1, P.Hlo[1] + j2, P.Hlo[2] + j3};
    // (2 pi i H_a)^k / k! per axis, in closed form
    if (lane < 3 * (N + 1)) {
        const int a = lane / (N + 1), k = lane % (N + 1);
        double mag = 1.0;
        const double t = 6.283185307179586476925 * (double)H[a];
        for (int i = 1; i <= k; ++i) mag *= t / i;
        const int ph = k & 3;    // i^k
        Ar[a][k] = ph == 0 ? mag : (ph == 2 ? -mag : 0.0);
        Ai[a][k] = ph == 1 ? mag : (ph == 3 ? -mag : 0.0);
    }
    for (int t = lane; t < T; t += 64)
        mono_s[t] = P.mono[3 * t] | (P.mono[3 * t + 1] << 8) | (P.mono[3 * t + 2] << 16);
    double s2 = 0.0;
    if (P.has_ff) {
        // |Q|-dependent scattering factor at Q = H (reciprocal-lattice units)
        double q[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) q[c] += H[a] * P.recip[3 * a + c];
        s2 = (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) / (16.0 * M_PI * M_PI);
    }
    for (int mu = lane; mu < P.S; mu += 64) {
        const auto* sd = gptr(P.site) + 12 * mu;
        double x = H[0] * sd[0] + H[1] * sd[1] + H[2] * sd[2];
        x -= floor(x);
        double sn, cs;
        sincos(6.283185307179586476925 * x, &sn, &cs);
        double wgt = sd[3];
        if (P.has_ff) {
            const auto* f = sd + 4;
            wgt *= f[0] * exp(-f[1] * s2) + f[2] * exp(-f[3] * s2) + f[4] * exp(-f[5] * s2) + f[6];
        }
        Wr[mu] = wgt * cs;
        Wi[mu] = wgt * sn;
    }
    __syncthreads();
    const int items = P.S * T;
    double sq = 0.0, mre = 0.0, mim = 0.0;
    for (int m = 0; m < P.M; ++m) {
        const auto* Sm = gptr(P.sums) + (size_t)m * items;    // [site][monomial] of configuration m
        double fr = 0.0, fi = 0.0;
#pragma unroll 4
        for (int it = lane; it < items; it += 64) {
            const int mu = it / T, t = it - mu * T;
            const int e = mono_s[t];
            const int p = e & 0xff, q = (e >> 8) & 0xff, r = e >> 16;
            const double xr = Ar[0][p] * Ar[1][q] - Ai[0][p] * Ai[1][q];
            const double xi = Ar[0][p] * Ai[1][q] + Ai[0][p] * Ar[1][q];
            const double sv = Sm[it];
            const double cr = (xr * Ar[2][r] - xi * Ai[2][r]) * sv;
            const double ci = (xr * Ai[2][r] + xi * Ar[2][r]) * sv;
            fr += cr * Wr[mu] - ci * Wi[mu];
            fi += cr * Wi[mu] + ci * Wr[mu];
        }
        for (int off = 32; off > 0; off >>= 1) {
            fr += __shfl_down(fr, off, 64);
            fi += __shfl_down(fi, off, 64);
        }
        sq += fr * fr + fi * fi;
        mre += fr; mim += fi;
    }
    if (lane == 0) {
        mre /= P.M; mim /= P.M;
        const double I = (sq / P.M - (mre * mre + mim * mim)) * P.scale;
        const int G[3] = {P.n[0] * H[0], P.n[1] * H[1], P.n[2] * H[2]};
        gptr(P.out)[((size_t)(G[0] - P.g0[0]) * P.cnt[1] + (G[1] - P.g0[1])) * P.opitch + (G[2] - P.g0[2]) + P.ooff] = (float)I;
    }
}

template <int N>
__global__ __launch_bounds__(64) void k_bragg_nuclear(BraggParams P) { bragg_nuclear_body<N, BraggParams>(P, blockIdx.x); }
template <int N>
__global__ __launch_bounds__(64) void k_bragg_nuclear_merged(const BraggParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) bragg_nuclear_body<N, const BraggParams&>(tab[d], bx);
}

// Taylor order 0 with few sites (one field per site, the occupancy): one lane per H.  The
// lane's site factors b_mu f(|H|) e^{2 pi i H.r_mu} are staged in its own LDS column, then
// every configuration is summed over the sites serially, so a wave serves 64 H where the
// form above, built for the many (site, monomial) pairs of a Taylor model, gives one H a wave.
constexpr int kBraggLaneSites = 16;

template <class PT>
__device__ __forceinline__ void bragg_lanes_body(PT P, const int bx)
{
#pragma clang fp contract(off)
    __shared__ double Wr[kBraggLaneSites][64], Wi[kBraggLaneSites][64];
    const int total = P.nH[0] * P.nH[1] * P.nH[2];
    const int lane = threadIdx.x;
    const int idx = bx * 64 + lane;
    if (idx >= total) return;                       // (no barrier below: each lane has its column)
    const int j3 = idx % P.nH[2], j2 = (idx / P.nH[2]) % P.nH[1], j1 = idx / (P.nH[2] * P.nH[1]);
    const int H[3] = {P.Hlo[0] + j1, P.Hlo[1] + j2, P.Hlo[2] + j3};
    double s2 = 0.0;
    if (P.has_ff) {
        double q[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) q[c] += H[a] * P.recip[3 * a + c];
        s2 = (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) / (16.0 * M_PI * M_PI);
    }
    for (int mu = 0; mu < P.S; ++mu) {
        const auto* sd = gptr(P.site) + 12 * mu;
        double x = H[0] * sd[0] + H[1] * sd[1] + H[2] * sd[2];
        x -= floor(x);
        double sn, cs;
        sincos(6.283185307179586476925 * x, &sn, &cs);
        double wgt = sd[3];
        if (P.has_ff) {
            const auto* f = sd + 4;
            wgt *= f[0] * exp(-f[1] * s2) + f[2] * exp(-f[3] * s2) + f[4] * exp(-f[5] * s2) + f[6];
        }
        Wr[mu][lane] = wgt * cs;
        Wi[mu][lane] = wgt * sn;
    }
    double sq = 0.0, mre = 0.0, mim = 0.0;
    for (int m = 0; m < P.M; ++m) {
        const auto* Sm = gptr(P.sums) + (size_t)m * P.S * P.T;   // [site][monomial]; monomial 0: occupancy
        double fr = 0.0, fi = 0.0;
        for (int mu = 0; mu < P.S; ++mu) {
            const double sv = Sm[(size_t)mu * P.T];
            fr += sv * Wr[mu][lane];
            fi += sv * Wi[mu][lane];
        }
        sq += fr * fr + fi * fi;
        mre += fr; mim += fi;
    }
    mre /= P.M; mim /= P.M;
    const double I = (sq / P.M - (mre * mre + mim * mim)) * P.scale;
    const int G[3] = {P.n[0] * H[0], P.n[1] * H[1], P.n[2] * H[2]};
    gptr(P.out)[((size_t)(G[0] - P.g0[0]) * P.cnt[1] + (G[1] - P.g0[1])) * P.opitch + (G[2] - P.g0[2]) + P.ooff] = (float)I;
}

__global__ __launch_bounds__(64) void k_bragg_lanes(BraggParams P) { bragg_lanes_body<BraggParams>(P, blockIdx.x); }
__global__ __launch_bounds__(64) void k_bragg_lanes_merged(const BraggParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) bragg_lanes_body<const BraggParams&>(tab[d], bx);
}

template <class FP>
__device__ double mag_ff_d(FP f, double s2) {
    return f[0] * exp(-f[1] * s2) + f[2] * exp(-f[3] * s2) + f[4] * exp(-f[5] * s2) + f[6];
}

// T_mu(H) of Eq. dw in float64: sum_t (2 pi i)^{p+q+r} H1^p H2^q H3^r / (p! q! r!) dwc[t].
__device__ void dw_at_h(const BraggParams& P, const int H[3], int mu, double& tr, double& ti)
{
    const double* c = P.dwc + (size_t)mu * P.dwT;
    tr = 0.0; ti = 0.0;
    for (int t = 0; t < P.dwT; ++t) {
        const int e[3] = {P.mono[3 * t], P.mono[3 * t + 1], P.mono[3 * t + 2]};
        double mag = c[t];
        for (int a = 0; a < 3; ++a)
            for (int k = 1; k <= e[a]; ++k) mag *= 6.283185307179586476925 * H[a] / k;
        switch ((e[0] + e[1] + e[2]) & 3) {
            case 0: tr += mag; break;
            case 1: ti += mag; break;
            case 2: tr -= mag; break;
            default: ti -= mag; break;
        }
    }
}

// One 64-lane wave per unit-cell Bragg point H: each lane forms, for its sites, the
// factor b_mu f_mu(|Q|) T_mu(H) e^{2 pi i H.r_mu} once, then per configuration the
// vector F = sum_mu factor S_mu (S the float64 lattice sums of the spins) is one wave
// reduction (fixed order); lane 0 projects F perpendicular to Q and keeps the ensemble
// moments.  All in float64.
template <class PT>
__device__ __forceinline__ void bragg_magnetic_body(PT P, const int bx)
{
    // every product and sum rounded on its own (no contraction into FMAs): the kernel and
    // its merged twin then compute the same bits, and the variance of one configuration
    // cancels to exactly 0
#pragma clang fp contract(off)
    __shared__ double Wr[4][kMaxSites], Wi[4][kMaxSites];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = bx * 4 + wave;
    const int total = P.nH[0] * P.nH[1] * P.nH[2];
    if (idx >= total) return;              // whole waves leave together; no block barrier follows
    const int j3 = idx % P.nH[2], j2 = (idx / P.nH[2]) % P.nH[1], j1 = idx / (P.nH[2] * P.nH[1]);
    const int H[3] = {P.Hlo[0] + j1, P.Hlo[1] + j2, P.Hlo[2] + j3};
    const int G[3] = {P.n[0] * H[0], P.n[1] * H[1], P.n[2] * H[2]};
    float* o = P.out + ((size_t)(G[0] - P.g0[0]) * P.cnt[1] + (G[1] - P.g0[1])) * P.opitch + (G[2] - P.g0[2]) + P.ooff;
    double Q[3];
    for (int c = 0; c < 3; ++c) Q[c] = H[0] * P.recip[c] + H[1] * P.recip[3 + c] + H[2] * P.recip[6 + c];
    const double q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
    if (!(q2 > 0.0)) {
        if (lane == 0) *o = 0.f;
        return;
    }
    const double s2 = q2 / (16.0 * 9.869604401089358618834);
    for (int mu = lane; mu < P.S; mu += 64) {
        const auto* sd = gptr(P.site) + 12 * mu;
        double x = H[0] * sd[0] + H[1] * sd[1] + H[2] * sd[2];
        x -= floor(x);
        double sn, cs;
        sincos(6.283185307179586476925 * x, &sn, &cs);
        const double f = P.has_ff ? mag_ff_d(sd + 4, s2) : 1.0;
        double wr = sd[3] * f * cs, wi = sd[3] * f * sn;
        if (P.dwc) {
            double tr, ti;
            dw_at_h(P, H, mu, tr, ti);
            const double xr = wr * tr - wi * ti;
            wi = wr * ti + wi * tr;
            wr = xr;
        }
        Wr[wave][mu] = wr;
        Wi[wave][mu] = wi;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const double iq = 1.0 / sqrt(q2);
    const double e[3] = {Q[0] * iq, Q[1] * iq, Q[2] * iq};
    double sq = 0.0, mr[3] = {0, 0, 0}, mi[3] = {0, 0, 0};
    for (int m = 0; m < P.M; ++m) {
        double fr[3] = {0, 0, 0}, fi[3] = {0, 0, 0};
        for (int mu = lane; mu < P.S; mu += 64) {
            const auto* Sm = gptr(P.sums) + ((size_t)m * P.S + mu) * 3;
            for (int c = 0; c < 3; ++c) {
                fr[c] += Sm[c] * Wr[wave][mu];
                fi[c] += Sm[c] * Wi[wave][mu];
            }
        }
        for (int off = 32; off > 0; off >>= 1)
            for (int c = 0; c < 3; ++c) {
                fr[c] += __shfl_down(fr[c], off, 64);
                fi[c] += __shfl_down(fi[c], off, 64);
            }
        if (lane == 0) {
            const double pr = e[0] * fr[0] + e[1] * fr[1] + e[2] * fr[2];
            const double pi = e[0] * fi[0] + e[1] * fi[1] + e[2] * fi[2];
            for (int c = 0; c < 3; ++c) {
                const double ar = fr[c] - e[c] * pr, ai = fi[c] - e[c] * pi;
                sq += ar * ar + ai * ai;
                mr[c] += ar; mi[c] += ai;
            }
        }
    }
    if (lane == 0) {
        double mm = 0.0;
        for (int c = 0; c < 3; ++c) {
            mr[c] /= P.M; mi[c] /= P.M;
            mm += mr[c] * mr[c] + mi[c] * mi[c];
        }
        *o = (float)((sq / P.M - mm) * P.scale);
    }
}

__global__ __launch_bounds__(256) void k_bragg_magnetic(BraggParams P) { bragg_magnetic_body<BraggParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_bragg_magnetic_merged(const BraggParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) bragg_magnetic_body<const BraggParams&>(tab[d], bx);
}

template <int N>
static hipError_t launch_bragg_t(const BraggParams& p, int grid, hipStream_t st)
{
    (void)grid;
    return dispatch(k_bragg_nuclear<N>, k_bragg_nuclear_merged<N>, p.nH[0] * p.nH[1] * p.nH[2], 64, 0, st, p);
}

hipError_t launch_bragg(const BraggParams& p, int order, hipStream_t st)
{
    const int total = p.nH[0] * p.nH[1] * p.nH[2];
    if (total <= 0) return hipSuccess;
    const int grid = (total + 255) / 256;
    if (p.kind == 1) {
        return dispatch(k_bragg_magnetic, k_bragg_magnetic_merged, (total + 3) / 4, 256, 0, st, p);
    }
    if (order == 0 && p.S <= kBraggLaneSites)
        return dispatch(k_bragg_lanes, k_bragg_lanes_merged, (total + 63) / 64, 64, 0, st, p);
    switch (order) {
        case 0: return launch_bragg_t<0>(p, grid, st);
        case 1: return launch_bragg_t<1>(p, grid, st);
        case 2: return launch_bragg_t<2>(p, grid, st);
        case 3: return launch_bragg_t<3>(p, grid, st);
        case 4: return launch_bragg_t<4>(p, grid, st);
        case 5: return launch_bragg_t<5>(p, grid, st);
        case 6: return launch_bragg_t<6>(p, grid, st);
        case 7: return launch_bragg_t<7>(p, grid, st);
        case 8: return launch_bragg_t<8>(p, grid, st);
        case 9: return launch_bragg_t<9>(p, grid, st);
        case 10: return launch_bragg_t<10>(p, grid, st);
        case 11: return launch_bragg_t<11>(p, grid, st);
        case 12: return launch_bragg_t<12>(p, grid, st);
        case 13: return launch_bragg_t<13>(p, grid, st);
        case 14: return launch_bragg_t<14>(p, grid, st);
        case 15: return launch_bragg_t<15>(p, grid, st);
        case 16: return launch_bragg_t<16>(p, grid, st);
        default: return hipErrorInvalidValue;
    }
}

// Debye-Waller means of Eq. dw: one thread per (site, monomial), configurations summed
// in order.
template <class PT>
__device__ __forceinline__ void dw_mean_body(PT P, const int bx)
{
    const int idx = bx * blockDim.x + threadIdx.x;
    if (idx >= P.S * P.T) return;
    const int mu = idx / P.T, t = idx - mu * P.T;
    double num = 0.0, den = 0.0;
    for (int m = 0; m < P.M; ++m) {
        const double* sm = P.sums + ((size_t)m * P.S + mu) * P.T;
        num += sm[t];
        den += sm[0];
    }
    P.dwc[idx] = den != 0.0 ? num / den : 0.0;
}

__global__ __launch_bounds__(256) void k_dw_mean(DwParams P) { dw_mean_body<DwParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_dw_mean_merged(const DwParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) dw_mean_body<const DwParams&>(tab[d], bx);
}

hipError_t launch_dw_mean(const DwParams& p, hipStream_t st)
{
    return dispatch(k_dw_mean, k_dw_mean_merged, (p.S * p.T + 255) / 256, 256, 0, st, p);
}

#endif  // DSX_RECOMBINE_PART

}  // namespace dsx
