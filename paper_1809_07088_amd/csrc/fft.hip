// Field generation, float64 lattice sums and the batched 3D real-to-complex FFT
// with the +i sign (X_k = sum_R x_R e^{+2 pi i k.R / n}), for gfx950.
//
//  k_sums        float64 sums S^{pqr}_{m,mu} = sum_R delta u1^p u2^q u3^r (nuclear) or
//                sum_R delta M_c (magnetic): the k = 0 coefficient of every field,
//                used for the Bragg points and to centre the float32 fields.
//  k_fft_planes  generates the real fields of one lattice plane R1 (the Taylor
//                monomials delta u1^p u2^q u3^r of Sec. III.C, the occupancy of Sec.
//                III.B or the spin components of Sec. III.D), minus their mean, and
//                transforms them along axes 3 (real-to-complex, two real rows packed
//                in one complex line) and 2, entirely in LDS.
//  k_fft_axis1   transforms along axis 1 in place, on LDS tiles of 64 contiguous
//                columns.
// The 1D transforms are Stockham auto-sort passes of radix 2, 3, 4, 5 and a direct
// DFT, one output per thread, for any other prime (planned first, where it needs no
// twiddles); twiddles come from a float64-generated table.
#include "dsx_internal.h"

namespace dsx {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }   // i a
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Quotient a / b for 0 <= a < 2^22 and 0 < b < 2^22, with rb ~= 1/b (float): the
// float estimate is off by at most one and is corrected with one remainder check.
__device__ __forceinline__ int qdiv(int a, int b, float rb)
{
    int q = (int)((float)a * rb);
    const int r = a - q * b;
    q += (r >= b) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

// One Stockham pass of radix R over nf x nlines lines of length n held in LDS.
// Element e of line l of batch b sits at base[b * fstride + l * lstride + e * estride].
// Ns is the product of the radices of the earlier passes.
__device__ void stockham_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                              int nlines, int lstride, int estride, int nf, int fstride,
                              int n, int R, int Ns, const float2* __restrict__ tw)
{
    const int nb = n / R;
    const int twstep = n / (Ns * R);
    const int total = nf * nlines * nb;
    const float rnb = 1.f / (float)nb, rnl = 1.f / (float)nlines, rns = 1.f / (float)Ns;
    if (R > 5) {
        // odd prime R: one output per work item, so a pass keeps every thread busy.
        // y_k = x'_0 + sum_{r=1}^{(R-1)/2} [(x'_r + x'_{R-r}) cos(2 pi r k / R)
        //                                   + i (x'_r - x'_{R-r}) sin(2 pi r k / R)],
        // x'_r = x_r e^{2 pi i r te / n} (te = 0 in the first pass).  r te <= R te < n
        // and r k mod R is stepped, so no index needs a division.
        const int step = n / R, h = (R - 1) / 2;
        const float rR = 1.f / (float)R;
        for (int it = threadIdx.x; it < total * R; it += blockDim.x) {
            const int B = qdiv(it, R, rR);
            const int k = it - B * R;
            const int L = qdiv(B, nb, rnb);
            const int j = B - L * nb;
            const int fb = qdiv(L, nlines, rnl), l = L - fb * nlines;
            const float2* x = src + fb * fstride + l * lstride + j * estride;
            const int jm = j - qdiv(j, Ns, rns) * Ns;
            const int o = (j - jm) * R + jm;
            const int te = jm * twstep;
            const int xs = nb * estride;
            float2 y = x[0];
            int b = 0;
            for (int r = 1; r <= h; ++r) {
                b += k;
                b -= (b >= R) ? R : 0;
                float2 xr = x[r * xs], xq = x[(R - r) * xs];
                if (Ns > 1) {
                    xr = cmul(xr, tw[r * te]);
                    xq = cmul(xq, tw[(R - r) * te]);
                }
                const float2 w = tw[b * step];
                const float2 sm = cadd(xr, xq), df = csub(xr, xq);
                y.x += sm.x * w.x - df.y * w.y;
                y.y += sm.y * w.x + df.x * w.y;
            }
            dst[fb * fstride + l * lstride + (o + k * Ns) * estride] = y;
        }
        return;
    }
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int L = qdiv(it, nb, rnb);
        const int j = it - L * nb;
        const int fb = qdiv(L, nlines, rnl), l = L - fb * nlines;
        const float2* s = src + fb * fstride + l * lstride;
        float2* d = dst + fb * fstride + l * lstride;
        const int jm = j - qdiv(j, Ns, rns) * Ns;
        const int o = (j - jm) * R + jm;          // (j / Ns) * Ns * R + j mod Ns
        const int te = jm * twstep;               // twiddle exponent step, r * te < n
        if (R == 4) {
            float2 v0 = s[j * estride];
            float2 v1 = cmul(s[(j + nb) * estride], tw[te]);
            float2 v2 = cmul(s[(j + 2 * nb) * estride], tw[2 * te]);
            float2 v3 = cmul(s[(j + 3 * nb) * estride], tw[3 * te]);
            float2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = cmuli(csub(v1, v3));
            d[o * estride] = cadd(a0, a2);
            d[(o + Ns) * estride] = cadd(a1, a3);
            d[(o + 2 * Ns) * estride] = csub(a0, a2);
            d[(o + 3 * Ns) * estride] = csub(a1, a3);
        } else if (R == 2) {
            float2 v0 = s[j * estride];
            float2 v1 = cmul(s[(j + nb) * estride], tw[te]);
            d[o * estride] = cadd(v0, v1);
            d[(o + Ns) * estride] = csub(v0, v1);
        } else if (R == 3) {
            const float h = 0.86602540378443864676f;   // sin(2 pi / 3)
            float2 v0 = s[j * estride];
            float2 v1 = cmul(s[(j + nb) * estride], tw[te]);
            float2 v2 = cmul(s[(j + 2 * nb) * estride], tw[2 * te]);
            float2 sm = cadd(v1, v2);
            float2 t = make_float2(v0.x - 0.5f * sm.x, v0.y - 0.5f * sm.y);
            float2 u = cscale(cmuli(csub(v1, v2)), h);
            d[o * estride] = cadd(v0, sm);
            d[(o + Ns) * estride] = cadd(t, u);
            d[(o + 2 * Ns) * estride] = csub(t, u);
        } else {   // R == 5
            const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
            const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
            float2 v0 = s[j * estride];
            float2 v1 = cmul(s[(j + nb) * estride], tw[te]);
            float2 v2 = cmul(s[(j + 2 * nb) * estride], tw[2 * te]);
            float2 v3 = cmul(s[(j + 3 * nb) * estride], tw[3 * te]);
            float2 v4 = cmul(s[(j + 4 * nb) * estride], tw[4 * te]);
            float2 b1 = cadd(v1, v4), b2 = cadd(v2, v3), d1 = csub(v1, v4), d2 = csub(v2, v3);
            float2 ra = make_float2(v0.x + c1 * b1.x + c2 * b2.x, v0.y + c1 * b1.y + c2 * b2.y);
            float2 rb = make_float2(v0.x + c2 * b1.x + c1 * b2.x, v0.y + c2 * b1.y + c1 * b2.y);
            float2 ia = cmuli(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
            float2 ib = cmuli(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
            d[o * estride] = make_float2(v0.x + b1.x + b2.x, v0.y + b1.y + b2.y);
            d[(o + Ns) * estride] = cadd(ra, ia);
            d[(o + 4 * Ns) * estride] = csub(ra, ia);
            d[(o + 2 * Ns) * estride] = cadd(rb, ib);
            d[(o + 3 * Ns) * estride] = csub(rb, ib);
        }
    }
}

// Full 1D transforms of all lines; ping-pongs between a and b and returns the
// buffer holding the result.  Caller synchronises before (inputs visible).
__device__ float2* lds_fft(float2* a, float2* b, int nlines, int lstride, int estride,
                           const AxisPlan& P, const float2* tw, int nf = 1, int fstride = 0)
{
    int Ns = 1;
    for (int s = 0; s < P.nrad; ++s) {
        stockham_pass(a, b, nlines, lstride, estride, nf, fstride, P.n, P.rad[s], Ns, tw);
        __syncthreads();
        Ns *= P.rad[s];
        float2* t = a; a = b; b = t;
    }
    return a;
}

// ---------------------------------------------------------------------------- sums
// Each thread walks P.chunk / 256 lattice cells and accumulates the monomials in
// groups of kSumsGroup float64 accumulators.  A group is reduced across the wave
// by recursive halving (each exchange moves half of the remaining values, so 32
// values need 32 exchanges instead of 32 x 6), then across the four waves through
// LDS.  The order of every addition is fixed: the sums are reproducible.
constexpr int kSumsGroup = 32;
constexpr int kSumsMaxPer = 8;    // cells per thread at most (the host's chunk is <= 8 x 256 cells)

template <int N>
struct MonoTable {
    int p[n_monomials(N)], q[n_monomials(N)], r[n_monomials(N)];
};

// (p, q, r) of every monomial index, in mono_index order
template <int N>
__host__ __device__ constexpr MonoTable<N> mono_table()
{
    MonoTable<N> m{};
    for (int dg = 0; dg <= N; ++dg)
        for (int p = dg; p >= 0; --p)
            for (int q = dg - p; q >= 0; --q) {
                const int t = mono_index(p, q, dg - p - q);
                m.p[t] = p; m.q[t] = q; m.r[t] = dg - p - q;
            }
    return m;
}

// One halving step: lanes with bit MASK set keep the upper HALF values, the others
// the lower HALF, each adding the partner's copy of the values it keeps.
template <int HALF, int MASK>
__device__ __forceinline__ void halve(double (&acc)[kSumsGroup], int lane)
{
    const bool hi = (lane & MASK) != 0;
#pragma unroll
    for (int k = 0; k < HALF; ++k) {
        const double send = hi ? acc[k] : acc[k + HALF];
        const double keep = hi ? acc[k + HALF] : acc[k];
        acc[k] = keep + __shfl_xor(send, MASK, 64);
    }
}

// Sum over the 64 lanes of acc[t] for every t; lane l (even) returns the total of
// acc[l >> 1].
__device__ __forceinline__ double wave_transpose_sum(double (&acc)[kSumsGroup], int lane)
{
    static_assert(kSumsGroup == 32, "five halving steps");
    halve<16, 32>(acc, lane);
    halve<8, 16>(acc, lane);
    halve<4, 8>(acc, lane);
    halve<2, 4>(acc, lane);
    halve<1, 2>(acc, lane);
    return acc[0] + __shfl_xor(acc[0], 1, 64);
}

template <int N, class PT>
__device__ __forceinline__ void sums_nuclear_body(PT P, const int bx)
{
    constexpr int T = n_monomials(N);
    constexpr MonoTable<N> mt = mono_table<N>();
    __shared__ double red[4][kSumsGroup];
    const int chunk = bx % P.nchunk;
    const int ms = bx / P.nchunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = chunk * P.chunk + threadIdx.x;
    const int c1 = min(P.ncell, (chunk + 1) * P.chunk);
    // this thread's cells (c0, c0 + 256, ...), loaded once for every monomial group;
    // the count is the same for the whole block
    const int ncl = (c1 - chunk * P.chunk + 255) / 256;
    float dv[kSumsMaxPer], uv[kSumsMaxPer][3];
#pragma unroll
    for (int i = 0; i < kSumsMaxPer; ++i) {
        const int c = c0 + 256 * i;
        const bool in = i < ncl && c < c1;
        const size_t at = (size_t)ms * P.ncell + (in ? c : 0);
        dv[i] = in ? (P.occ ? gptr(P.occ)[at] : 1.f) : 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) uv[i][a] = (in && N > 0 && P.vec) ? gptr(P.vec)[3 * at + a] : 0.f;
    }
    // orders above kMaxOrderFast keep the group loop rolled (up to 31 groups of 32)
    constexpr int kGroupUnroll = N <= kMaxOrderFast ? 8 : 1;
#pragma unroll kGroupUnroll
    for (int g0 = 0; g0 < T; g0 += kSumsGroup) {
        double acc[kSumsGroup];
#pragma unroll
        for (int t = 0; t < kSumsGroup; ++t) acc[t] = 0.0;
#pragma unroll
        for (int i = 0; i < kSumsMaxPer; ++i) {
            if (i >= ncl) break;
            const double d = (double)dv[i];
            double pw[3][N + 1];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                pw[a][0] = 1.0;
                const double u = (double)uv[i][a];
#pragma unroll
                for (int k = 1; k <= N; ++k) pw[a][k] = pw[a][k - 1] * u;
            }
#pragma unroll
            for (int t = 0; t < kSumsGroup; ++t)
                if (g0 + t < T)
                    acc[t] += d * pw[0][mt.p[g0 + t]] * pw[1][mt.q[g0 + t]] * pw[2][mt.r[g0 + t]];
        }
        const double v = wave_transpose_sum(acc, lane);
        if ((lane & 1) == 0) red[wave][lane >> 1] = v;
        __syncthreads();
        if (threadIdx.x < kSumsGroup && g0 + (int)threadIdx.x < T) {
            const int t = threadIdx.x;
            P.partial[((size_t)ms * P.nchunk + chunk) * T + g0 + t] =
                (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
        }
        __syncthreads();
    }
}

template <int N>
__global__ __launch_bounds__(256) void k_sums_nuclear(SumsParams P) { sums_nuclear_body<N, SumsParams>(P, blockIdx.x); }
template <int N>
__global__ __launch_bounds__(256) void k_sums_nuclear_merged(const SumsParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) sums_nuclear_body<N, const SumsParams&>(tab[d], bx);
}

template <class PT>
__device__ __forceinline__ void sums_magnetic_body(PT P, const int bx)
{
    __shared__ double red[4][3];
    const int chunk = bx % P.nchunk;
    const int ms = bx / P.nchunk;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[3] = {0.0, 0.0, 0.0};
    const int c0 = chunk * P.chunk;
    const int c1 = min(P.ncell, c0 + P.chunk);
    for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const size_t at = (size_t)ms * P.ncell + c;
        const double d = P.occ ? (double)gptr(P.occ)[at] : 1.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a] += d * (double)gptr(P.vec)[3 * at + a];
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        double v = acc[t];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wave][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
        P.partial[((size_t)ms * P.nchunk + chunk) * 3 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(256) void k_sums_magnetic(SumsParams P) { sums_magnetic_body<SumsParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_sums_magnetic_merged(const SumsParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) sums_magnetic_body<const SumsParams&>(tab[d], bx);
}

// One wave per output sum: lanes read the chunk partials, then a fixed-order
// shuffle reduction (reproducible).
template <class PT>
__device__ __forceinline__ void sums_reduce_body(PT P, const int bx)
{
    const int idx = bx * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (idx >= P.M * P.S * P.T) return;
    const int ms = idx / P.T, t = idx - ms * P.T;
    double v = 0.0;
    for (int c = lane; c < P.nchunk; c += 64) v += P.partial[((size_t)ms * P.nchunk + c) * P.T + t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) gptr(P.sums)[idx] = v;
}

__global__ __launch_bounds__(256) void k_sums_reduce(SumsParams P) { sums_reduce_body<SumsParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_sums_reduce_merged(const SumsParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) sums_reduce_body<const SumsParams&>(tab[d], bx);
}

template <int N>
static hipError_t launch_sums_t(const SumsParams& p, hipStream_t st)
{
    return dispatch(k_sums_nuclear<N>, k_sums_nuclear_merged<N>, p.M * p.S * p.nchunk, 256, 0, st, p);
}

hipError_t launch_sums(const SumsParams& p, int order, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (p.kind == 1) {
        e = dispatch(k_sums_magnetic, k_sums_magnetic_merged, p.M * p.S * p.nchunk, 256, 0, st, p);
    } else {
        switch (order) {
            case 0: e = launch_sums_t<0>(p, st); break;
            case 1: e = launch_sums_t<1>(p, st); break;
            case 2: e = launch_sums_t<2>(p, st); break;
            case 3: e = launch_sums_t<3>(p, st); break;
            case 4: e = launch_sums_t<4>(p, st); break;
            case 5: e = launch_sums_t<5>(p, st); break;
            case 6: e = launch_sums_t<6>(p, st); break;
            case 7: e = launch_sums_t<7>(p, st); break;
            case 8: e = launch_sums_t<8>(p, st); break;
            case 9: e = launch_sums_t<9>(p, st); break;
            case 10: e = launch_sums_t<10>(p, st); break;
            case 11: e = launch_sums_t<11>(p, st); break;
            case 12: e = launch_sums_t<12>(p, st); break;
            case 13: e = launch_sums_t<13>(p, st); break;
            case 14: e = launch_sums_t<14>(p, st); break;
            case 15: e = launch_sums_t<15>(p, st); break;
            case 16: e = launch_sums_t<16>(p, st); break;
            default: return hipErrorInvalidValue;
        }
    }
    if (e != hipSuccess) return e;
    const int tot = p.M * p.S * p.T;
    return dispatch(k_sums_reduce, k_sums_reduce_merged, (tot + 3) / 4, 256, 0, st, p);
}

// ---------------------------------------------------------------------------- plane FFT
// Generates the nfb fields fa.. of rows 2 j0 .. 2 (j0 + nj) - 1 of the npl lattice planes
// R1 .. R1 + npl - 1 of site mu, configuration m (centred by their float64 mean), packs two
// real rows per complex line, transforms the lines along axis 3 in LDS and separates the
// two half spectra.  Item b = pl nfb + fb is field fa + fb of plane R1 + pl.  Returns the
// LDS buffer holding row r (local) of item b at [b * BE + r * nh + k3]; A and B are
// ping-pong buffers of npl nfb x BE elements.
__device__ __forceinline__ float2* planes_rows(const PlaneParams& P, float2* A, float2* B, const float2* tw3, int m, int mu,
                               int R1, int npl, int j0, int nj, int fa, int nfb, int BE)
{
    const int n2 = P.n2, n3 = P.n3, nh = P.nh;
    const int ncell = P.n1 * n2 * n3;
    const size_t plane0 = ((size_t)(m * P.S + mu)) * ncell + (size_t)R1 * n2 * n3;
    const auto* occ0 = P.occ ? gptr(P.occ) + plane0 : nullptr;
    const auto* vec0 = P.vec ? gptr(P.vec) + 3 * plane0 : nullptr;
    const float rpn3 = 1.f / (float)(nj * n3), rn3 = 1.f / (float)n3, rnh = 1.f / (float)nh;
    const float rpnh = 1.f / (float)(nj * nh), rnfb = 1.f / (float)nfb;
    const int nb = npl * nfb;
    for (int idx = threadIdx.x; idx < nb * nj * n3; idx += blockDim.x) {
        const int b = qdiv(idx, nj * n3, rpn3);
        const int rem = idx - b * nj * n3;
        const int jj = qdiv(rem, n3, rn3), R3 = rem - jj * n3;
        const int pl = qdiv(b, nfb, rnfb), fb = b - pl * nfb;
        const auto* occ = occ0 ? occ0 + (size_t)pl * n2 * n3 : nullptr;
        const auto* vec = vec0 ? vec0 + (size_t)3 * pl * n2 * n3 : nullptr;
        const int f = fa + fb;
        const int ep = P.mono[3 * f], eq = P.mono[3 * f + 1], er = P.mono[3 * f + 2];
        const int t = P.kind == 1 ? f : mono_index(ep, eq, er);    // index of the field's lattice sum
        const float mean = (float)(gptr(P.sums)[(size_t)(m * P.S + mu) * P.T + t] / (double)ncell);
        float xv[2] = {0.f, 0.f};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int R2 = 2 * (j0 + jj) + h;
            if (R2 < n2) {
                const int c = R2 * n3 + R3;
                float v;
                if (P.kind == 1) {
                    v = vec[3 * c + t];
                } else {
                    v = 1.f;
                    if (ep | eq | er) {
                        const float u0 = vec[3 * c], u1 = vec[3 * c + 1], u2 = vec[3 * c + 2];
                        for (int k = 0; k < ep; ++k) v *= u0;
                        for (int k = 0; k < eq; ++k) v *= u1;
                        for (int k = 0; k < er; ++k) v *= u2;
                    }
                }
                if (occ) v *= occ[c];
                xv[h] = v - mean;
            }
        }
        A[b * BE + jj * n3 + R3] = make_float2(xv[0], xv[1]);
    }
    __syncthreads();
    float2* Z = lds_fft(A, B, nj, n3, 1, P.p3, tw3, nb, BE);
    float2* C = (Z == A) ? B : A;
    // unpack the packed real transforms: X_a = (Z_k + conj Z_-k)/2, X_b = -i (Z_k - conj Z_-k)/2
    for (int idx = threadIdx.x; idx < nb * nj * nh; idx += blockDim.x) {
        const int b = qdiv(idx, nj * nh, rpnh);
        const int rem = idx - b * nj * nh;
        const int jj = qdiv(rem, nh, rnh), k = rem - jj * nh;
        const float2 zk = Z[b * BE + jj * n3 + k];
        const int km = (k == 0) ? 0 : n3 - k;
        const float2 zm = Z[b * BE + jj * n3 + km];
        const float2 xa = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 xb = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
        C[b * BE + (2 * jj) * nh + k] = xa;
        if (2 * (j0 + jj) + 1 < n2) C[b * BE + (2 * jj + 1) * nh + k] = xb;
    }
    __syncthreads();
    return C;
}

template <class PT>
__device__ __forceinline__ void fft_planes_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    float2* tw2 = smem;
    float2* tw3 = tw2 + P.n2;
    float2* A = tw3 + P.n3;
    float2* B = A + P.npl * P.fchunk * P.buf_elems;

    int b = bx;
    const int fc = b % P.nfchunk; b /= P.nfchunk;
    const int nrb = (P.n1 + P.npl - 1) / P.npl;      // plane blocks per (site, configuration)
    const int R1 = (b % nrb) * P.npl; b /= nrb;
    const int mu = b % P.S;
    const int m = b / P.S;
    const int n2 = P.n2, nh = P.nh;
    const int SF = P.S * P.F;

    for (int i = threadIdx.x; i < n2; i += blockDim.x) tw2[i] = ldg2(P.tw2, i);
    for (int i = threadIdx.x; i < P.n3; i += blockDim.x) tw3[i] = ldg2(P.tw3, i);
    const int fa = fc * P.fchunk;
    const int nfb = min(P.F, fa + P.fchunk) - fa;     // fields of this block, batched
    const int npl = min(P.npl, P.n1 - R1);            // and planes
    const int BE = P.buf_elems;
    __syncthreads();   // twiddles visible
    float2* C = planes_rows(P, A, B, tw3, m, mu, R1, npl, 0, (n2 + 1) / 2, fa, nfb, BE);
    float2* D = (C == A) ? B : A;
    float2* Y = lds_fft(C, D, nh, 1, nh, P.p2, tw2, npl * nfb, BE);
    // write: for each plane and k2, the block's fields are contiguous runs of nh complex
    const float rnh = 1.f / (float)nh, rfnh = 1.f / (float)(nfb * nh), rpl = 1.f / (float)(n2 * nfb * nh);
    float2* out = P.X + ((size_t)(m * P.n1 + R1) * n2) * SF * nh + (size_t)(mu * P.F + fa) * nh;
    for (int idx = threadIdx.x; idx < npl * n2 * nfb * nh; idx += blockDim.x) {
        const int pl = qdiv(idx, n2 * nfb * nh, rpl);
        const int r2 = idx - pl * n2 * nfb * nh;
        const int k2 = qdiv(r2, nfb * nh, rfnh);
        const int rem = r2 - k2 * nfb * nh;
        const int fb = qdiv(rem, nh, rnh), k3 = rem - fb * nh;
        stg2(out, ((size_t)pl * n2 + k2) * SF * nh + rem, Y[(pl * nfb + fb) * BE + k2 * nh + k3]);
    }
}

__global__ __launch_bounds__(256) void k_fft_planes(PlaneParams P) { fft_planes_body<PlaneParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_fft_planes_merged(const PlaneParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) fft_planes_body<const PlaneParams&>(tab[d], bx);
}

// Planes that do not fit the LDS: rows 2 j0 .. of a plane (P.row_pairs pairs per block)
// generated and transformed along axis 3 only, written with the row index R2 in place
// of k2; the axis-2 transform then runs in place like the axis-1 one.
template <class PT>
__device__ __forceinline__ void fft_rows_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    float2* tw3 = smem;
    float2* A = tw3 + P.n3;
    float2* B = A + P.fchunk * P.buf_elems;
    int b = bx;
    const int fc = b % P.nfchunk; b /= P.nfchunk;
    const int rc = b % P.nrchunk; b /= P.nrchunk;
    const int R1 = b % P.n1; b /= P.n1;
    const int mu = b % P.S;
    const int m = b / P.S;
    const int n2 = P.n2, nh = P.nh;
    const int SF = P.S * P.F;
    for (int i = threadIdx.x; i < P.n3; i += blockDim.x) tw3[i] = ldg2(P.tw3, i);
    const int fa = fc * P.fchunk;
    const int nfb = min(P.F, fa + P.fchunk) - fa;
    const int j0 = rc * P.row_pairs;
    const int nj = min((n2 + 1) / 2, j0 + P.row_pairs) - j0;
    const int BE = P.buf_elems;
    __syncthreads();
    const float2* C = planes_rows(P, A, B, tw3, m, mu, R1, 1, j0, nj, fa, nfb, BE);
    const int nrow = min(n2, 2 * (j0 + nj)) - 2 * j0;
    const float rnh = 1.f / (float)nh, rfnh = 1.f / (float)(nfb * nh);
    float2* out = P.X + ((size_t)(m * P.n1 + R1) * n2 + 2 * j0) * SF * nh + (size_t)(mu * P.F + fa) * nh;
    for (int idx = threadIdx.x; idx < nrow * nfb * nh; idx += blockDim.x) {
        const int r = qdiv(idx, nfb * nh, rfnh);
        const int rem = idx - r * nfb * nh;
        const int fb = qdiv(rem, nh, rnh), k3 = rem - fb * nh;
        stg2(out, (size_t)r * SF * nh + rem, C[fb * BE + r * nh + k3]);
    }
}

__global__ __launch_bounds__(256) void k_fft_rows(PlaneParams P) { fft_rows_body<PlaneParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_fft_rows_merged(const PlaneParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) fft_rows_body<const PlaneParams&>(tab[d], bx);
}

// ---------------------------------------------------------------------------- register FFTs
// Power-of-two lengths L <= 32 are transformed by one thread in registers
// (radix-2 decimation in time, input in bit-reversed order), so a line needs no
// LDS passes and no barriers.
__host__ __device__ constexpr int bit_reverse(int i, int L)
{
    int r = 0;
    for (int b = 1; b < L; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
    return r;
}

template <int L>
__device__ __forceinline__ void fft_reg(float2 (&z)[L], const float2* __restrict__ tw)   // tw[t] = e^{+2 pi i t / L}
{
#pragma unroll
    for (int st = 0; (1 << st) < L; ++st) {
        const int half = 1 << st;
        const int step = L / (2 * half);
#pragma unroll
        for (int k = 0; k < L; k += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const float2 a = z[k + j];
                float2 b = z[k + j + half];
                if (j * step == L / 4) b = cmuli(b);          // e^{+i pi / 2} = i
                else if (j != 0) b = cmul(b, tw[j * step]);
                z[k + j] = cadd(a, b);
                z[k + j + half] = csub(a, b);
            }
        }
    }
}

// Axis 1 in place: one thread per column (k2, c), the L1 values of the column in
// registers.  Columns are contiguous in memory, so every load and store of a wave
// is one contiguous run.
template <int L1, class PT>
__device__ __forceinline__ void fft_axis1_reg_body(PT P, const int bx)
{
    __shared__ float2 tw[L1];
    for (int i = threadIdx.x; i < L1; i += blockDim.x) tw[i] = ldg2(P.tw1, i);
    __syncthreads();
    const unsigned per_m = (unsigned)P.n2 * (unsigned)P.cols;
    const unsigned g = bx * blockDim.x + threadIdx.x;
    if (g >= per_m * (unsigned)P.M) return;
    const unsigned m = g / per_m, rem = g - m * per_m;
    float2* base = P.X + (size_t)m * L1 * per_m + rem;
    float2 z[L1];
#pragma unroll
    for (int i = 0; i < L1; ++i) z[i] = ldg2(base, (size_t)bit_reverse(i, L1) * per_m);
    fft_reg<L1>(z, tw);
#pragma unroll
    for (int k = 0; k < L1; ++k) stg2(base, (size_t)k * per_m, z[k]);
}

template <int L1>
__global__ __launch_bounds__(256) void k_fft_axis1_reg(Axis1Params P) { fft_axis1_reg_body<L1, Axis1Params>(P, blockIdx.x); }
template <int L1>
__global__ __launch_bounds__(256) void k_fft_axis1_reg_merged(const Axis1Params* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) fft_axis1_reg_body<L1, const Axis1Params&>(tab[d], bx);
}

// One lattice plane R1 of one site, a chunk of kRegFC fields, for power-of-two
// n2 = L2, n3 = L3 <= 32:
//  1. every thread generates the chunk's fields of a few cells (the powers of a
//     p-run are stepped by one factor u_1 each), centred by the FP64 mean, into LDS;
//  2. one thread per (field, row pair) packs two real rows into one complex line and
//     transforms it along axis 3 in registers, then separates the two half spectra;
//  3. one thread per (field, k3) transforms the column along axis 2 in registers and
//     writes it to the spectra (k3 fastest across the wave: contiguous runs).
constexpr int kRegFC = 8, kRegThreads = 128;

template <int L2, int L3, class PT>
__device__ __forceinline__ void fft_planes_reg_body(PT P, const int bx)
{
    constexpr int NH = L3 / 2 + 1;
    constexpr int RP = L3 + 1;                         // real row pitch (floats)
    constexpr int FS = ((L2 * RP + 31) / 32) * 32 + 1; // real field stride: lanes of two fields hit other banks
    constexpr int CP = L2 + 1;                         // complex column pitch
    constexpr int CS = NH * CP;                        // complex field stride
    constexpr int UN = (kRegFC * FS > 2 * kRegFC * CS) ? kRegFC * FS : 2 * kRegFC * CS;   // floats
    __shared__ float2 tw2[L2], tw3[L3];
    __shared__ float buf[UN];
    __shared__ float meanf[kRegFC];

    int b = bx;
    const int fc = b % P.nfchunk; b /= P.nfchunk;
    const int R1 = b % P.n1; b /= P.n1;
    const int mu = b % P.S;
    const int m = b / P.S;
    const int ncell = P.n1 * L2 * L3;
    const int fa = fc * kRegFC;
    const int nfb = min(P.F, fa + kRegFC) - fa;
    for (int i = threadIdx.x; i < L2; i += blockDim.x) tw2[i] = ldg2(P.tw2, i);
    for (int i = threadIdx.x; i < L3; i += blockDim.x) tw3[i] = ldg2(P.tw3, i);
    if (threadIdx.x < nfb) {
        const int f = fa + threadIdx.x;
        const int ep = P.mono[3 * f], eq = P.mono[3 * f + 1], er = P.mono[3 * f + 2];
        const int t = P.kind == 1 ? f : mono_index(ep, eq, er);
        meanf[threadIdx.x] = (float)(gptr(P.sums)[(size_t)(m * P.S + mu) * P.T + t] / (double)ncell);
    }
    __syncthreads();

    // 1. generation.  The thread's cells are loaded together (one memory latency);
    //    the loop over the chunk's fields is uniform, so exponents are scalars and a
    //    field continuing the p-run of the previous one costs one product per cell.
    const size_t plane0 = ((size_t)(m * P.S + mu)) * ncell + (size_t)R1 * L2 * L3;
    static_assert(kRegThreads % L3 == 0, "a thread's cells share r3");
    constexpr int CPT = (L2 * L3 + kRegThreads - 1) / kRegThreads;   // cells per thread
    constexpr int RSTEP = kRegThreads / L3;            // rows between a thread's cells
    const bool gen = threadIdx.x < L2 * L3;           // false only on planes under kRegThreads cells
    float cd[CPT], cu0[CPT], cu1[CPT], cu2[CPT], v[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const size_t c = plane0 + threadIdx.x + k * kRegThreads;
        cd[k] = (gen && P.occ) ? gptr(P.occ)[c] : 1.f;
        cu0[k] = cu1[k] = cu2[k] = 0.f;
        if (gen && P.vec) {
            const auto* u = gptr(P.vec) + 3 * c;
            cu0[k] = u[0]; cu1[k] = u[1]; cu2[k] = u[2];
        }
        v[k] = 1.f;
    }
    float* const dst0 = buf + (threadIdx.x / L3) * RP + threadIdx.x % L3;
    int pe = -1, qe = -1, re = -1;                     // exponents of the previous field
    for (int fb = 0; fb < (gen ? nfb : 0); ++fb) {
        const int f = fa + fb;
        const float mf = meanf[fb];
        float* const dst = dst0 + fb * FS;
        if (P.kind == 1) {
#pragma unroll
            for (int k = 0; k < CPT; ++k)
                dst[k * RSTEP * RP] = (f == 0 ? cu0[k] : f == 1 ? cu1[k] : cu2[k]) * cd[k] - mf;
            continue;
        }
        const int ep = P.mono[3 * f], eq = P.mono[3 * f + 1], er = P.mono[3 * f + 2];
        if (ep == pe + 1 && eq == qe && er == re) {
#pragma unroll
            for (int k = 0; k < CPT; ++k) v[k] *= cu0[k];
        } else {
#pragma unroll
            for (int k = 0; k < CPT; ++k) v[k] = 1.f;
            for (int e = 0; e < ep; ++e)
#pragma unroll
                for (int k = 0; k < CPT; ++k) v[k] *= cu0[k];
            for (int e = 0; e < eq; ++e)
#pragma unroll
                for (int k = 0; k < CPT; ++k) v[k] *= cu1[k];
            for (int e = 0; e < er; ++e)
#pragma unroll
                for (int k = 0; k < CPT; ++k) v[k] *= cu2[k];
        }
        pe = ep; qe = eq; re = er;
#pragma unroll
        for (int k = 0; k < CPT; ++k) dst[k * RSTEP * RP] = v[k] * cd[k] - mf;
    }
    __syncthreads();

    // 2. axis 3: two real rows per complex line, then the two half spectra
    constexpr int NP = L2 / 2;
    const int t = threadIdx.x;
    const int fb3 = t / NP, j = t - fb3 * NP;
    const bool act3 = t < kRegFC * NP && fb3 < nfb;
    float2 z[L3];
    if (act3) {
        const float* r0 = buf + fb3 * FS + (2 * j) * RP;
#pragma unroll
        for (int i = 0; i < L3; ++i) z[i] = make_float2(r0[bit_reverse(i, L3)], r0[RP + bit_reverse(i, L3)]);
        fft_reg<L3>(z, tw3);
    }
    __syncthreads();                      // the real rows are no longer needed
    float2* cb = reinterpret_cast<float2*>(buf);
    if (act3) {
        float2* col = cb + fb3 * CS + 2 * j;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const float2 zk = z[k], zm = z[(L3 - k) % L3];
            col[k * CP] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            col[k * CP + 1] = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
        }
    }
    __syncthreads();

    // 3. axis 2, written to the spectra
    const int SF = P.S * P.F;
    float2* out = P.X + ((size_t)(m * P.n1 + R1) * L2) * SF * NH + (size_t)(mu * P.F + fa) * NH;
    for (int it = threadIdx.x; it < nfb * NH; it += blockDim.x) {
        const int fb = it / NH, k = it - fb * NH;
        const float2* col = cb + fb * CS + k * CP;
        float2 y[L2];
#pragma unroll
        for (int i = 0; i < L2; ++i) y[i] = col[bit_reverse(i, L2)];
        fft_reg<L2>(y, tw2);
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) stg2(out, (size_t)k2 * SF * NH + it, y[k2]);
    }
}

template <int L2, int L3>
__global__ __launch_bounds__(kRegThreads) void k_fft_planes_reg(PlaneParams P) { fft_planes_reg_body<L2, L3, PlaneParams>(P, blockIdx.x); }
template <int L2, int L3>
__global__ __launch_bounds__(kRegThreads) void k_fft_planes_reg_merged(const PlaneParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) fft_planes_reg_body<L2, L3, const PlaneParams&>(tab[d], bx);
}

bool fft_reg_supported(int n) { return n == 8 || n == 16 || n == 32; }

template <int L2, int L3>
static hipError_t launch_planes_reg(const PlaneParams& p, hipStream_t st)
{
    PlaneParams q = p;
    q.fchunk = kRegFC;
    q.nfchunk = (p.F + kRegFC - 1) / kRegFC;
    return dispatch(k_fft_planes_reg<L2, L3>, k_fft_planes_reg_merged<L2, L3>, q.M * q.S * q.n1 * q.nfchunk,
                    kRegThreads, 0, st, q);
}

template <int L2>
static hipError_t launch_planes_reg2(const PlaneParams& p, hipStream_t st)
{
    switch (p.n3) {
        case 8: return launch_planes_reg<L2, 8>(p, st);
        case 16: return launch_planes_reg<L2, 16>(p, st);
        case 32: return launch_planes_reg<L2, 32>(p, st);
        default: return hipErrorInvalidValue;
    }
}

size_t planes_lds_bytes(const PlaneParams& p)
{
    return sizeof(float2) * (size_t)((p.row_pairs > 0 ? 0 : p.n2) + p.n3 + 2 * (p.npl > 1 ? p.npl : 1) * p.fchunk * p.buf_elems);
}

hipError_t launch_fft_planes(const PlaneParams& p, hipStream_t st)
{
    if (fft_reg_supported(p.n2) && fft_reg_supported(p.n3)) {
        switch (p.n2) {
            case 8: return launch_planes_reg2<8>(p, st);
            case 16: return launch_planes_reg2<16>(p, st);
            default: return launch_planes_reg2<32>(p, st);
        }
    }
    const size_t lds = planes_lds_bytes(p);
    if (p.row_pairs > 0) {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)k_fft_rows,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        return dispatch(k_fft_rows, k_fft_rows_merged, p.M * p.S * p.n1 * p.nrchunk * p.nfchunk, 256, lds, st, p);
    }
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_fft_planes,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (p.npl < 1) return hipErrorInvalidValue;
    return dispatch(k_fft_planes, k_fft_planes_merged, p.M * p.S * ((p.n1 + p.npl - 1) / p.npl) * p.nfchunk, 256, lds,
                    st, p);
}

// ---------------------------------------------------------------------------- axis-1 FFT
template <class PT>
__device__ __forceinline__ void fft_axis1_body(PT P, const int bx)
{
    extern __shared__ float2 smem[];
    float2* tw = smem;
    float2* A = tw + P.n1;
    float2* B = A + P.n1 * P.tc;
    int b = bx;
    const int cb = b % P.ncolblk; b /= P.ncolblk;
    const int k2 = b % P.n2;
    const int m = b / P.n2;
    const int tc = P.tc, n1 = P.n1;
    const int c0 = cb * tc;
    const size_t rowstride = (size_t)P.n2 * P.cols;
    float2* base = P.X + ((size_t)m * n1 * P.n2 + k2) * P.cols + c0;
    for (int i = threadIdx.x; i < n1; i += blockDim.x) tw[i] = ldg2(P.tw1, i);
    for (int b0 = threadIdx.x; b0 < n1 * tc; b0 += 8 * blockDim.x) {
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = b0 + u * blockDim.x;
            const int R1 = idx / tc, c = idx - R1 * tc;
            v[u] = (idx < n1 * tc && c0 + c < P.cols) ? ldg2(base, R1 * rowstride + c) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = b0 + u * blockDim.x;
            if (idx < n1 * tc) A[idx] = v[u];
        }
    }
    __syncthreads();
    float2* Y = lds_fft(A, B, tc, 1, tc, P.p1, tw);
    for (int idx = threadIdx.x; idx < n1 * tc; idx += blockDim.x) {
        const int k1 = idx / tc, c = idx - k1 * tc;
        if (c0 + c < P.cols) stg2(base, k1 * rowstride + c, Y[idx]);
    }
}

__global__ __launch_bounds__(256) void k_fft_axis1(Axis1Params P) { fft_axis1_body<Axis1Params>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_fft_axis1_merged(const Axis1Params* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) fft_axis1_body<const Axis1Params&>(tab[d], bx);
}

size_t axis1_lds_bytes(const Axis1Params& p)
{
    return sizeof(float2) * (size_t)(p.n1 + 2 * p.n1 * p.tc);
}

hipError_t launch_fft_axis1(const Axis1Params& p, hipStream_t st)
{
    if (fft_reg_supported(p.n1)) {
        const unsigned total = (unsigned)p.M * p.n2 * p.cols;
        const unsigned grid = (total + 255) / 256;
        if (p.n1 == 8) return dispatch(k_fft_axis1_reg<8>, k_fft_axis1_reg_merged<8>, grid, 256, 0, st, p);
        if (p.n1 == 16) return dispatch(k_fft_axis1_reg<16>, k_fft_axis1_reg_merged<16>, grid, 256, 0, st, p);
        return dispatch(k_fft_axis1_reg<32>, k_fft_axis1_reg_merged<32>, grid, 256, 0, st, p);
    }
    const size_t lds = axis1_lds_bytes(p);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_fft_axis1,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return dispatch(k_fft_axis1, k_fft_axis1_merged, p.M * p.n2 * p.ncolblk, 256, lds, st, p);
}

}  // namespace dsx
