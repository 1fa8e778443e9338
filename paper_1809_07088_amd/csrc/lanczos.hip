// Lanczos (windowed-sinc) resampling of I(G) for gfx950 (Sec. V.B, Eqs.
// intensity_convol_finite, windowed_sinc, lanczos).
//
// The weight W(Q - G) is a product over the axes and the window takes the 2m
// points floor(Q_a) - m + 1 <= G_a <= floor(Q_a) + m on every axis, so the
// normalised sum  sum_G I(G) W / sum_G W  equals three normalised 1D passes, one
// per axis, applied in sequence (the paper notes this separability).  The weights,
// normalised per output phase i mod s, come from a float64 host table.
//
// One block owns an output tile T2 x T3 and a segment of T1 outputs along axis 1.
// It streams the input planes e1 of that segment once: each plane is staged in
// LDS (rows and halo), filtered along axis 3 then axis 2, and kept in a ring of
// 2m filtered planes; an output plane is emitted as soon as its 2m input planes
// are in the ring.  Every input value is read from HBM about once per block.
#include "dsx_internal.h"

namespace dsx {

// Tile of block b: blocks are dealt round-robin to the 8 XCDs, so XCD x is given
// the x-th contiguous eighth of the tiles and neighbouring tiles (which share halo
// rows and output cache lines) meet in one L2.  Returns -1 past the last tile.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    const int per = (ntiles + 7) / 8;
    const int t = (b % 8) * per + b / 8;
    return t < ntiles ? t : -1;
}

template <class PT>
__device__ __forceinline__ void lanczos_body(PT P, const int bx)
{
    extern __shared__ float sm[];
    const int m2 = 2 * P.m, s = P.s;
    int b = xcd_tile(bx, P.nb1 * P.nb2 * P.nb3);
    if (b < 0) return;
    const int b3 = b % P.nb3; b /= P.nb3;
    const int b2 = b % P.nb2;
    const int b1 = b / P.nb2;
    const int o1 = b1 * P.t1, o2 = b2 * P.t2, o3 = b3 * P.t3;
    const int T1 = min(P.t1, P.o[0] - o1), T2 = min(P.t2, P.o[1] - o2), T3 = min(P.t3, P.o[2] - o3);
    const int eo = P.eoff;
    const int E2lo = o2 / s + eo, E2n = (o2 + T2 - 1) / s + eo - E2lo + m2;
    const int E3lo = o3 / s + eo, E3n = (o3 + T3 - 1) / s + eo - E3lo + m2;
    const int L2max = (P.t2 - 1) / s + 1 + m2, L3max = (P.t3 - 1) / s + 1 + m2;

    float* wn = sm;                                  // [s][2m]
    float* stg = wn + ((s * m2 + 3) & ~3);           // [E2n][E3n]
    float* mid = stg + L2max * L3max;                // [E2n][t3]
    float* ring = mid + L2max * P.t3;                // [2m][t2][t3]
    for (int i = threadIdx.x; i < s * m2; i += blockDim.x) wn[i] = P.wn[i];

    const int tile = P.t2 * P.t3;
    const int e1a = o1 / s + eo, e1b = (o1 + T1 - 1) / s + eo + m2 - 1;
    for (int e1 = e1a; e1 <= e1b; ++e1) {
        __syncthreads();
        const bool mir = e1 >= P.ihalf;
        const size_t pbase = (size_t)(mir ? P.e[0] - 1 - e1 : e1) * P.e[1];
        for (int idx = threadIdx.x; idx < E2n * E3n; idx += blockDim.x) {
            const int r = idx / E3n, c = idx - r * E3n;
            int row = E2lo + r, colx = E3lo + c;
            if (mir) { row = P.e[1] - 1 - row; colx = P.e[2] - 1 - colx; }
            stg[idx] = P.in[P.ioff + (pbase + row) * P.ipitch + colx];
        }
        __syncthreads();
        // axis 3
        for (int idx = threadIdx.x; idx < E2n * T3; idx += blockDim.x) {
            const int r = idx / T3, j3 = idx - r * T3;
            const int i3 = o3 + j3;
            const float* w = wn + (i3 % s) * m2;
            const float* x = stg + r * E3n + (i3 / s + eo - E3lo);
            float acc = 0.f;
            for (int d = 0; d < m2; ++d) acc += w[d] * x[d];
            mid[r * P.t3 + j3] = acc;
        }
        __syncthreads();
        // axis 2 into the ring slot of plane e1
        float* slot = ring + (e1 % m2) * tile;
        for (int idx = threadIdx.x; idx < T2 * T3; idx += blockDim.x) {
            const int j2 = idx / T3, j3 = idx - j2 * T3;
            const int i2 = o2 + j2;
            const float* w = wn + (i2 % s) * m2;
            const float* x = mid + (i2 / s + eo - E2lo) * P.t3 + j3;
            float acc = 0.f;
            for (int d = 0; d < m2; ++d) acc += w[d] * x[d * P.t3];
            slot[j2 * P.t3 + j3] = acc;
        }
        __syncthreads();
        // axis 1: outputs whose window ends at plane e1
        const int fl = e1 - m2 + 1;       // first input plane of the window
        if (fl >= e1a) {
            const int ia = max(o1, (fl - eo) * s), ib = min(o1 + T1, (fl - eo) * s + s);
            for (int i1 = ia; i1 < ib; ++i1) {
                const float* w = wn + (i1 % s) * m2;
                float* orow = P.out + ((size_t)i1 * P.o[1] + o2) * P.o[2] + o3;
                for (int idx = threadIdx.x; idx < T2 * T3; idx += blockDim.x) {
                    const int j2 = idx / T3, j3 = idx - j2 * T3;
                    float acc = 0.f;
                    for (int d = 0; d < m2; ++d)
                        acc += w[d] * ring[((fl + d) % m2) * tile + j2 * P.t3 + j3];
                    orow[(size_t)j2 * P.o[2] + j3] = acc;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_lanczos(LanczosParams P) { lanczos_body<LanczosParams>(P, blockIdx.x); }
__global__ __launch_bounds__(256) void k_lanczos_merged(const LanczosParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) lanczos_body<const LanczosParams&>(tab[d], bx);
}

// Register-ring variant for m = M2/2 in {2, 3, 4} and a 32 x 64 output tile.
// Per input plane: the plane's tile (with halo) is staged in LDS; the axis-3 pass
// gives each thread a run of four consecutive columns of one row (it reads the
// M2 + 3 inputs of the run once); the axis-2 pass gives each thread four
// consecutive rows of one column, whose filtered values join a register ring of
// the last M2 planes; the axis-1 pass then emits the thread's four outputs of the
// plane whose window is complete.  The next two input planes are in flight in
// registers while a plane is filtered.  Three block barriers per plane.
constexpr int kRT2 = 32, kRT3 = 64, kRThreads = 512, kRRun = 4;

template <int M2, bool S1, class PT>
__device__ __forceinline__ void lanczos_ring_body(PT P, const int bx)
{
    constexpr int L2 = kRT2 + M2 - 1;                     // staged rows (s = 1)
    constexpr int L3 = (kRT3 + M2 - 1 + 3) & ~3;          // staged row pitch (s = 1), 16-byte rows
    constexpr int NSTG = (L2 * L3 + kRThreads - 1) / kRThreads;
    __shared__ float wn_s[16 * M2];
    __shared__ __align__(16) float stg[(S1 ? L2 * L3 : 1)];
    __shared__ __align__(16) float mid[(S1 ? L2 * kRT3 : 1)];
    static_assert(S1, "the oversampled filter takes the generic kernel");
    int b = xcd_tile(bx, P.nb1 * P.nb2 * P.nb3);
    if (b < 0) return;
    const int b3 = b % P.nb3; b /= P.nb3;
    const int b2 = b % P.nb2;
    const int b1 = b / P.nb2;
    const int eo = P.eoff;
    // column tiles are cut at multiples of 64 in input coordinates (o3 + eo)
    const int o1 = b1 * P.t1, o2 = b2 * kRT2, o3 = max(0, b3 * kRT3 - eo);
    const int T1 = min(P.t1, (P.ohalf ? P.ohalf : P.o[0]) - o1), T2 = min(kRT2, P.o[1] - o2);
    const int T3 = min((b3 + 1) * kRT3 - eo, P.o[2]) - o3;
    const int E2lo = o2 + eo, E2n = T2 + M2 - 1;
    const int E3lo = o3 + eo, E3n = T3 + M2 - 1;
    for (int i = threadIdx.x; i < M2; i += blockDim.x) wn_s[i] = gptr(P.wn)[i];

    // this thread's staging elements (row-major, pitch L3), as offsets within a stored
    // plane and within the mirrored plane (rows and columns reversed)
    int soff[NSTG], moff[NSTG];
#pragma unroll
    for (int k = 0; k < NSTG; ++k) {
        const int idx = threadIdx.x + kRThreads * k;
        const int r = idx / L3, c = idx - r * L3;
        const bool in = idx < L2 * L3 && r < E2n && c < E3n;
        soff[k] = in ? (E2lo + r) * P.ipitch + E3lo + c + P.ioff : -1;
        moff[k] = in ? (P.e[1] - 1 - E2lo - r) * P.ipitch + (P.e[2] - 1 - E3lo - c) + P.ioff : -1;
    }
    const size_t plane = (size_t)P.e[1] * P.ipitch;
    const int e1a = o1 + eo, e1b = o1 + T1 - 1 + eo + M2 - 1;
    auto fetch = [&](int e1, float (&buf)[NSTG]) {
        const bool mir = e1 >= P.ihalf;
        const auto* src = gptr(P.in) + (size_t)(mir ? P.e[0] - 1 - e1 : e1) * plane;
#pragma unroll
        for (int k = 0; k < NSTG; ++k)
            if (soff[k] >= 0) buf[k] = src[mir ? moff[k] : soff[k]];
    };
    float pa[NSTG], pb[NSTG];
#pragma unroll
    for (int k = 0; k < NSTG; ++k) pa[k] = pb[k] = 0.f;
    fetch(e1a, pa);
    if (e1a + 1 <= e1b) fetch(e1a + 1, pb);
    // axis-2 / axis-1 ownership: column j3, rows 4 g .. 4 g + 3
    const int j3 = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    float ring[M2][kRRun];
#pragma unroll
    for (int d = 0; d < M2; ++d)
#pragma unroll
        for (int k = 0; k < kRRun; ++k) ring[d][k] = 0.f;
    float w[M2];

    auto plane_step = [&](int e1, float (&buf)[NSTG]) {
        __syncthreads();                      // the previous plane's staging is consumed
#pragma unroll
        for (int k = 0; k < NSTG; ++k) {
            const int idx = threadIdx.x + kRThreads * k;
            if (idx < L2 * L3) stg[idx] = buf[k];
        }
        if (e1 + 2 <= e1b) fetch(e1 + 2, buf);
        __syncthreads();
#pragma unroll
        for (int d = 0; d < M2; ++d) w[d] = wn_s[d];
        // axis 3: runs of four columns
        for (int t = threadIdx.x; t < E2n * (kRT3 / kRRun); t += kRThreads) {
            const int r = t / (kRT3 / kRRun), c0 = (t - r * (kRT3 / kRRun)) * kRRun;
            const float* x = stg + r * L3 + c0;
            float xv[kRRun + M2 - 1];
#pragma unroll
            for (int i = 0; i < kRRun + M2 - 1; ++i) xv[i] = x[i];
            float4 o;
            float* op = reinterpret_cast<float*>(&o);
#pragma unroll
            for (int q = 0; q < kRRun; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int d = 0; d < M2; ++d) acc += w[d] * xv[q + d];
                op[q] = acc;
            }
            *reinterpret_cast<float4*>(mid + r * kRT3 + c0) = o;
        }
        __syncthreads();
        // axis 2: four consecutive rows of column j3 into the ring (shift by one plane)
        float xv[kRRun + M2 - 1];
#pragma unroll
        for (int i = 0; i < kRRun + M2 - 1; ++i) {
            const int r = g * kRRun + i;
            xv[i] = r < E2n ? mid[r * kRT3 + j3] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < kRRun; ++q) {
            float v = 0.f;
#pragma unroll
            for (int d = 0; d < M2; ++d) v += w[d] * xv[q + d];
#pragma unroll
            for (int d = 0; d < M2 - 1; ++d) ring[d][q] = ring[d + 1][q];
            ring[M2 - 1][q] = v;
        }
        // axis 1: the output plane whose window ends at input plane e1
        const int i1 = e1 - M2 + 1 - eo;
        if (i1 >= o1 && j3 < T3) {
            auto* orow = gptr(P.out) + ((size_t)i1 * P.o[1] + o2) * P.o[2] + o3 + j3;
            // the mirrored output (-G): plane o0 - 1 - i1, rows and columns reversed
            const bool mirror = P.ohalf && i1 != P.o[0] - 1 - i1;
            auto* mrow = gptr(P.out) + ((size_t)(P.o[0] - 1 - i1) * P.o[1] + (P.o[1] - 1 - o2)) * P.o[2]
                        + (P.o[2] - 1 - o3 - j3);
#pragma unroll
            for (int q = 0; q < kRRun; ++q) {
                const int j2 = g * kRRun + q;
                if (j2 < T2) {
                    float acc = 0.f;
#pragma unroll
                    for (int d = 0; d < M2; ++d) acc += w[d] * ring[d][q];
                    orow[(size_t)j2 * P.o[2]] = acc;
                    if (mirror) mrow[-(ptrdiff_t)j2 * P.o[2]] = acc;
                }
            }
        }
    };
    for (int e1 = e1a; e1 <= e1b; e1 += 2) {
        plane_step(e1, pa);
        if (e1 + 1 <= e1b) plane_step(e1 + 1, pb);
    }
}

template <int M2, bool S1>
__global__ __launch_bounds__(512, 2) void k_lanczos_ring(LanczosParams P) { lanczos_ring_body<M2, S1, LanczosParams>(P, blockIdx.x); }
template <int M2, bool S1>
__global__ __launch_bounds__(512, 2) void k_lanczos_ring_merged(const LanczosParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) lanczos_ring_body<M2, S1, const LanczosParams&>(tab[d], bx);
}

size_t lanczos_lds_bytes(const LanczosParams& p)
{
    const int m2 = 2 * p.m;
    const int L2max = (p.t2 - 1) / p.s + 1 + m2, L3max = (p.t3 - 1) / p.s + 1 + m2;
    return sizeof(float) * (size_t)(((p.s * m2 + 3) & ~3) + L2max * L3max + L2max * p.t3 +
                                    m2 * p.t2 * p.t3);
}

bool lanczos_ring_supported(const LanczosParams& p)
{
    return p.s == 1 && (p.m == 2 || p.m == 3 || p.m == 4);
}

hipError_t launch_lanczos(const LanczosParams& p, hipStream_t st)
{
    if (lanczos_ring_supported(p)) {
        LanczosParams q = p;
        q.t2 = kRT2; q.t3 = kRT3;
        q.nb2 = (p.o[1] + kRT2 - 1) / kRT2;
        q.nb3 = (p.o[2] + p.eoff + kRT3 - 1) / kRT3;
        if (p.ohalf) q.nb1 = (p.ohalf + p.t1 - 1) / p.t1;
        const unsigned grid = 8 * ((q.nb1 * q.nb2 * q.nb3 + 7) / 8);
        if (p.m == 2) return dispatch(k_lanczos_ring<4, true>, k_lanczos_ring_merged<4, true>, grid, kRThreads, 0, st, q);
        if (p.m == 3) return dispatch(k_lanczos_ring<6, true>, k_lanczos_ring_merged<6, true>, grid, kRThreads, 0, st, q);
        return dispatch(k_lanczos_ring<8, true>, k_lanczos_ring_merged<8, true>, grid, kRThreads, 0, st, q);
    }
    const size_t lds = lanczos_lds_bytes(p);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_lanczos,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return dispatch(k_lanczos, k_lanczos_merged, 8 * ((p.nb1 * p.nb2 * p.nb3 + 7) / 8), 256, lds, st, p);
}

// ---------------------------------------------------------------------------- points
// The windowed sum at arbitrary points (off-axis planes such as (h h l), any grid):
// one thread per point forms the 2w one-axis weights of each axis (float, from the
// float64 offsets Q_a - G_a), then sums the (2w)^3 neighbourhood from the dense box,
// which the host sized to hold every window.  The normaliser is the product of the
// three one-axis weight sums (the weight is separable).
template <int W, class PT>
__device__ __forceinline__ void lanczos_points_body(PT P, const int bx)
{
    const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
    if (i >= P.npts) return;
    float wt[3][2 * W];
    int lo[3];
    float norm = 1.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double Q = P.q[3 * i + a];
        const double f = floor(Q);
        lo[a] = (int)f - W + 1 - P.e0[a];
        float sum = 0.f;
#pragma unroll
        for (int t = 0; t < 2 * W; ++t) {
            const float d = (float)(Q - (f - W + 1 + t));      // Q_a - G_a
            float v = 0.f;
            if (fabsf(d) < (float)W) {
                const float x1 = 6.283185307179586f * P.rcut * d, x2 = 3.141592653589793f * d / (float)W;
                v = (x1 == 0.f ? 1.f : sinf(x1) / x1) * (x2 == 0.f ? 1.f : sinf(x2) / x2);
            }
            wt[a][t] = v;
            sum += v;
        }
        norm *= sum;
    }
    const size_t p2 = (size_t)P.e[2], p1 = (size_t)P.e[1] * P.e[2];
    float acc = 0.f;
    for (int t1 = 0; t1 < 2 * W; ++t1) {
        const float* plane = P.in + (size_t)(lo[0] + t1) * p1;
        float a1 = 0.f;
#pragma unroll
        for (int t2 = 0; t2 < 2 * W; ++t2) {
            const float* row = plane + (size_t)(lo[1] + t2) * p2 + lo[2];
            float a2 = 0.f;
#pragma unroll
            for (int t3 = 0; t3 < 2 * W; ++t3) a2 = fmaf(wt[2][t3], row[t3], a2);
            a1 = fmaf(wt[1][t2], a2, a1);
        }
        acc = fmaf(wt[0][t1], a1, acc);
    }
    P.out[i] = acc / norm;
}

template <int W>
__global__ __launch_bounds__(256) void k_lanczos_points(PointsParams P) { lanczos_points_body<W, PointsParams>(P, blockIdx.x); }
template <int W>
__global__ __launch_bounds__(256) void k_lanczos_points_merged(const PointsParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) lanczos_points_body<W, const PointsParams&>(tab[d], bx);
}

hipError_t launch_lanczos_points(const PointsParams& p, hipStream_t st)
{
    const unsigned grid = (unsigned)((p.npts + 255) / 256);
    switch (p.w) {
        case 1: return dispatch(k_lanczos_points<1>, k_lanczos_points_merged<1>, grid, 256, 0, st, p);
        case 2: return dispatch(k_lanczos_points<2>, k_lanczos_points_merged<2>, grid, 256, 0, st, p);
        case 3: return dispatch(k_lanczos_points<3>, k_lanczos_points_merged<3>, grid, 256, 0, st, p);
        case 4: return dispatch(k_lanczos_points<4>, k_lanczos_points_merged<4>, grid, 256, 0, st, p);
        case 5: return dispatch(k_lanczos_points<5>, k_lanczos_points_merged<5>, grid, 256, 0, st, p);
        case 6: return dispatch(k_lanczos_points<6>, k_lanczos_points_merged<6>, grid, 256, 0, st, p);
        case 7: return dispatch(k_lanczos_points<7>, k_lanczos_points_merged<7>, grid, 256, 0, st, p);
        case 8: return dispatch(k_lanczos_points<8>, k_lanczos_points_merged<8>, grid, 256, 0, st, p);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------- spherical
// The spherical cutoff makes the weight non-separable, so each output takes the
// whole (2m)^3 neighbourhood: one thread per output voxel, consecutive lanes on
// consecutive i3 (every tap's loads are one contiguous run, served from L2).  The
// normalised weights of the s^3 output phases come from a float64 host table
// [s^3][(2m)^3]; the input is the grown box, mirrored planes read as in the ring
// filter.
template <int T, class PT>
__device__ __forceinline__ void lanczos_stencil_body(PT P, const int bx)
{
    const int64_t idx = (int64_t)bx * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)P.o[0] * P.o[1] * P.o[2];
    if (idx >= total) return;
    const int i3 = (int)(idx % P.o[2]);
    const int i2 = (int)((idx / P.o[2]) % P.o[1]);
    const int i1 = (int)(idx / ((int64_t)P.o[2] * P.o[1]));
    const int s = P.s;
    const int phase = ((i1 % s) * s + (i2 % s)) * s + (i3 % s);
    const float* w = P.wn + (size_t)phase * T * T * T;
    const int b1 = i1 / s + P.eoff, b2 = i2 / s + P.eoff, b3 = i3 / s + P.eoff;
    const size_t plane = (size_t)P.e[1] * P.ipitch;
    float acc = 0.f;
    for (int t1 = 0; t1 < T; ++t1) {
        const int e1 = b1 + t1;
        const bool mir = e1 >= P.ihalf;
        const float* pl = P.in + (size_t)(mir ? P.e[0] - 1 - e1 : e1) * plane + P.ioff;
#pragma unroll
        for (int t2 = 0; t2 < T; ++t2) {
            const int e2 = mir ? P.e[1] - 1 - (b2 + t2) : b2 + t2;
            const float* row = pl + (size_t)e2 * P.ipitch;
#pragma unroll
            for (int t3 = 0; t3 < T; ++t3) {
                const int e3 = mir ? P.e[2] - 1 - (b3 + t3) : b3 + t3;
                acc = fmaf(w[(t1 * T + t2) * T + t3], row[e3], acc);
            }
        }
    }
    P.out[idx] = acc;
}

template <int T>
__global__ __launch_bounds__(256) void k_lanczos_stencil(LanczosParams P) { lanczos_stencil_body<T, LanczosParams>(P, blockIdx.x); }
template <int T>
__global__ __launch_bounds__(256) void k_lanczos_stencil_merged(const LanczosParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) lanczos_stencil_body<T, const LanczosParams&>(tab[d], bx);
}

// s = 1: every output has the same weights.  A block stages the input tile of a
// 4 x 8 x 64 output tile (with its halo) in LDS, and each thread computes the eight
// outputs (i1, i2 = 0..7, i3) of its column: every staged row feeds the outputs of
// all the i2 it reaches, so an output costs about T (T + 7) / 8 LDS reads instead
// of T^3 loads.
constexpr int kSt1 = 4, kSt2 = 8, kSt3 = 64;
template <int T, class PT>
__device__ __forceinline__ void lanczos_stencil_tile_body(PT P, const int bx)
{
    constexpr int A = kSt1 + T - 1, B = kSt2 + T - 1, C = kSt3 + T - 1;
    constexpr int CP = C + 1;                                  // LDS row pitch
    __shared__ float tile[A * B * CP];
    const int nb3 = (P.o[2] + kSt3 - 1) / kSt3, nb2 = (P.o[1] + kSt2 - 1) / kSt2;
    int b = bx;
    const int bx3 = b % nb3; b /= nb3;
    const int bx2 = b % nb2;
    const int bx1 = b / nb2;
    const int o1 = bx1 * kSt1, o2 = bx2 * kSt2, o3 = bx3 * kSt3;
    const size_t plane = (size_t)P.e[1] * P.ipitch;
    // stage: element (a, y, c) is input (o1 + eoff + a, o2 + eoff + y, o3 + eoff + c)
    for (int k = threadIdx.x; k < A * B * C; k += blockDim.x) {
        const int c = k % C, r = k / C;
        const int y = r % B, a = r / B;
        const int e1 = o1 + P.eoff + a, e2 = o2 + P.eoff + y, e3 = o3 + P.eoff + c;
        float v = 0.f;
        if (e1 < P.e[0] && e2 < P.e[1] && e3 < P.e[2]) {
            const bool mir = e1 >= P.ihalf;
            const size_t off = mir ? (size_t)(P.e[0] - 1 - e1) * plane + (size_t)(P.e[1] - 1 - e2) * P.ipitch
                                         + (P.e[2] - 1 - e3)
                                   : (size_t)e1 * plane + (size_t)e2 * P.ipitch + e3;
            v = P.in[off + P.ioff];
        }
        tile[(a * B + y) * CP + c] = v;
    }
    __syncthreads();
    const int c3 = threadIdx.x & 63, g = threadIdx.x >> 6;      // i3 lane, i1 within the tile
    float acc[kSt2] = {};
#pragma unroll 1
    for (int t1 = 0; t1 < T; ++t1) {
        const float* pl = tile + (size_t)((g + t1) * B) * CP + c3;
#pragma unroll
        for (int y = 0; y < B; ++y) {
            float x[T];
#pragma unroll
            for (int t3 = 0; t3 < T; ++t3) x[t3] = pl[y * CP + t3];
#pragma unroll
            for (int t2 = 0; t2 < T; ++t2) {
                const int q = y - t2;                           // output i2 this row reaches
                if (q >= 0 && q < kSt2) {
                    const float* w = P.wn + (t1 * T + t2) * T;
#pragma unroll
                    for (int t3 = 0; t3 < T; ++t3) acc[q] = fmaf(w[t3], x[t3], acc[q]);
                }
            }
        }
    }
    const int i1 = o1 + g, i3 = o3 + c3;
    if (i1 < P.o[0] && i3 < P.o[2]) {
        float* o = P.out + ((size_t)i1 * P.o[1] + o2) * P.o[2] + i3;
#pragma unroll
        for (int q = 0; q < kSt2; ++q)
            if (o2 + q < P.o[1]) o[(size_t)q * P.o[2]] = acc[q];
    }
}

template <int T>
__global__ __launch_bounds__(256) void k_lanczos_stencil_tile(LanczosParams P) { lanczos_stencil_tile_body<T, LanczosParams>(P, blockIdx.x); }
template <int T>
__global__ __launch_bounds__(256) void k_lanczos_stencil_tile_merged(const LanczosParams* __restrict__ tab, const Slot* __restrict__ slots)
{
    int d, bx;
    if (slot_of(slots, d, bx)) lanczos_stencil_tile_body<T, const LanczosParams&>(tab[d], bx);
}

hipError_t launch_lanczos_stencil(const LanczosParams& p, hipStream_t st)
{
    if (p.s == 1) {
        const unsigned grid = (unsigned)(((p.o[0] + kSt1 - 1) / kSt1) * ((p.o[1] + kSt2 - 1) / kSt2) *
                                         ((p.o[2] + kSt3 - 1) / kSt3));
        switch (2 * p.m) {
            case 4: return dispatch(k_lanczos_stencil_tile<4>, k_lanczos_stencil_tile_merged<4>, grid, 256, 0, st, p);
            case 6: return dispatch(k_lanczos_stencil_tile<6>, k_lanczos_stencil_tile_merged<6>, grid, 256, 0, st, p);
            case 8: return dispatch(k_lanczos_stencil_tile<8>, k_lanczos_stencil_tile_merged<8>, grid, 256, 0, st, p);
            default: return hipErrorInvalidValue;
        }
    }
    const int64_t total = (int64_t)p.o[0] * p.o[1] * p.o[2];
    const unsigned grid = (unsigned)((total + 255) / 256);
    switch (2 * p.m) {
        case 4: return dispatch(k_lanczos_stencil<4>, k_lanczos_stencil_merged<4>, grid, 256, 0, st, p);
        case 6: return dispatch(k_lanczos_stencil<6>, k_lanczos_stencil_merged<6>, grid, 256, 0, st, p);
        case 8: return dispatch(k_lanczos_stencil<8>, k_lanczos_stencil_merged<8>, grid, 256, 0, st, p);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dsx
