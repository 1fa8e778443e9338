/*
 * FP64 CPU oracle for the diffuse-scattering hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its binding) never links, loads or calls it, and the two
 * share no code.
 *
 * Everything here is the plain definition, written out as a direct summation
 * over atoms in double precision, parallelised over output points with OpenMP:
 *
 *   orc_sf_nuclear   F_m(G) = sum_{R,mu} b_mu delta e^{2 pi i g.(R + r_mu + u)}
 *                    (Sec. II, Eq. sf; Sec. III.A, Eq. total_sf), with g = G/n in
 *                    reciprocal-lattice units (Eq. G_def).  exact mode evaluates
 *                    e^{i G.u} directly; order-N mode replaces it by its Taylor
 *                    polynomial sum_{k<=N} (i G.u)^k / k! (Sec. III.C, Eq.
 *                    disp_expansion, with G.u = 2 pi sum_alpha g_alpha u^alpha,
 *                    Eq. gdotu_1).
 *   orc_sf_magnetic  vector F_m(G) = sum_{R,mu} b_mu delta M e^{2 pi i g.(R + r_mu)}
 *                    per site (Sec. III.D, Eqs. mag_sf, mag_ft); the form factor, the
 *                    Debye-Waller factor, the perpendicular projection and the
 *                    constant are applied by the Python side.
 *   orc_dw_mean      the Debye-Waller factor T_mu(G) of Sec. III.A, Eq. dw: the mean of
 *                    e^{i G.u} over the occupied atoms of a site, every cell and every
 *                    configuration (exact or order-N Taylor polynomial).
 *   orc_subbox       the method of sub-boxes of Sec. V.A: every lattice point the origin of
 *                    an open-boundary sub-box, |F|^2 and F averaged over origins and
 *                    configurations at arbitrary Q (the slow reference the Lanczos filter
 *                    of Sec. V.B is compared with).
 *   orc_pair_sum     (1/N) sum_{j,k} b_j b_k e^{i Q.(r_j - r_k)} with the
 *                    nearest-image convention (Sec. II, Eq. intensity_dble_sum).
 *   orc_lanczos      the windowed-sinc resampling of Sec. V.B (Eqs.
 *                    intensity_convol_finite, windowed_sinc, weight_sinc, lanczos)
 *                    summed directly over the (2m)^3 neighbourhood, NOT separably;
 *                    orc_lanczos_cutoff the same with the cutoff of the m' modification
 *                    (Sec. V.B, the second of the three modifications), and
 *                    orc_lanczos_points at arbitrary Q (not on the s-grid), and
 *                    orc_lanczos_spherical with the spherically symmetric cutoff W_r
 *                    (the third modification) in place of Eq. weight_sinc.
 *
 * The lattice-point part of every phase is reduced exactly in integers first:
 * e^{2 pi i G_a R_a / n_a} = e^{2 pi i ((G_a R_a) mod n_a) / n_a}.  This is an
 * identity, done only so that the double-precision argument stays small.
 *
 * Error behaviour: every entry point returns 0 on success and -1 on a bad
 * argument; outputs are written only on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586476925286766559

static long imodl(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }

static int bad_dims(const int32_t* n) { return n[0] < 1 || n[1] < 1 || n[2] < 1; }

/* Structure factor of a nuclear model (see file header).
 * n[3]        supercell
 * S           number of species-sites
 * frac[S][3]  average fractional positions r_mu (unit-cell coordinates)
 * b[S]        scattering lengths
 * M           number of configurations
 * occ         [M][S][n1][n2][n3] occupancy or NULL (= 1)
 * disp        [M][S][n1][n2][n3][3] fractional displacements or NULL (= 0)
 * order       < 0: exact exponential; >= 0: Taylor polynomial of that order
 * nG, G       [nG][3] integer supercell Bragg indices
 * F           [M][nG][2] output (re, im)
 */
int orc_sf_nuclear(const int32_t* n, int32_t S, const double* frac, const double* b,
                   int32_t M, const float* occ, const float* disp, int32_t order,
                   int64_t nG, const int32_t* G, double* F)
{
    if (bad_dims(n) || S < 1 || M < 1 || nG < 0 || !frac || !b || !G || !F) return -1;
    const long n1 = n[0], n2 = n[1], n3 = n[2];
    const long ncell = n1 * n2 * n3;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t gi = 0; gi < nG; ++gi) {
        const long G1 = G[3 * gi], G2 = G[3 * gi + 1], G3 = G[3 * gi + 2];
        const double g[3] = {(double)G1 / n1, (double)G2 / n2, (double)G3 / n3};
        for (int32_t m = 0; m < M; ++m) {
            double fr = 0.0, fi = 0.0;
            for (int32_t mu = 0; mu < S; ++mu) {
                const double gr = g[0] * frac[3 * mu] + g[1] * frac[3 * mu + 1] + g[2] * frac[3 * mu + 2];
                for (long R1 = 0; R1 < n1; ++R1)
                for (long R2 = 0; R2 < n2; ++R2)
                for (long R3 = 0; R3 < n3; ++R3) {
                    const long cell = (R1 * n2 + R2) * n3 + R3;
                    const long at = ((long)m * S + mu) * ncell + cell;
                    const double delta = occ ? (double)occ[at] : 1.0;
                    const double lat = (double)imodl(G1 * R1, n1) / n1 + (double)imodl(G2 * R2, n2) / n2
                                     + (double)imodl(G3 * R3, n3) / n3;
                    double gu = 0.0;
                    if (disp) {
                        const float* u = disp + 3 * at;
                        gu = g[0] * u[0] + g[1] * u[1] + g[2] * u[2];
                    }
                    double er, ei;
                    if (order < 0) {
                        const double ph = TWO_PI * (lat + gr + gu);
                        er = cos(ph); ei = sin(ph);
                    } else {
                        /* e^{2 pi i (lat + gr)} * sum_{k=0}^{order} (i x)^k / k!,  x = 2 pi g.u */
                        const double ph = TWO_PI * (lat + gr);
                        const double x = TWO_PI * gu;
                        double sr = 0.0, si = 0.0, tr = 1.0, ti = 0.0;
                        for (int k = 0; k <= order; ++k) {
                            sr += tr; si += ti;
                            /* t <- t * (i x) / (k + 1) */
                            const double nr = -ti * x / (k + 1), ni = tr * x / (k + 1);
                            tr = nr; ti = ni;
                        }
                        const double c = cos(ph), s = sin(ph);
                        er = c * sr - s * si; ei = c * si + s * sr;
                    }
                    fr += b[mu] * delta * er;
                    fi += b[mu] * delta * ei;
                }
            }
            F[2 * ((int64_t)m * nG + gi)] = fr;
            F[2 * ((int64_t)m * nG + gi) + 1] = fi;
        }
    }
    return 0;
}

/* Vector structure factor of a magnetic model, per site, without form factor
 * (see header).  The per-site split lets the caller apply a different form factor
 * to each site before summing.
 * spin [M][S][n1][n2][n3][3] Cartesian moments; occ optional as above.
 * F    [M][nG][S][3][2] output:  sum_R b_mu delta M e^{2 pi i g.(R + r_mu)}. */
int orc_sf_magnetic(const int32_t* n, int32_t S, const double* frac, const double* b,
                    int32_t M, const float* occ, const float* spin,
                    int64_t nG, const int32_t* G, double* F)
{
    if (bad_dims(n) || S < 1 || M < 1 || nG < 0 || !frac || !b || !spin || !G || !F) return -1;
    const long n1 = n[0], n2 = n[1], n3 = n[2];
    const long ncell = n1 * n2 * n3;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t gi = 0; gi < nG; ++gi) {
        const long G1 = G[3 * gi], G2 = G[3 * gi + 1], G3 = G[3 * gi + 2];
        const double g[3] = {(double)G1 / n1, (double)G2 / n2, (double)G3 / n3};
        for (int32_t m = 0; m < M; ++m) {
            for (int32_t mu = 0; mu < S; ++mu) {
                double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
                const double gr = g[0] * frac[3 * mu] + g[1] * frac[3 * mu + 1] + g[2] * frac[3 * mu + 2];
                for (long R1 = 0; R1 < n1; ++R1)
                for (long R2 = 0; R2 < n2; ++R2)
                for (long R3 = 0; R3 < n3; ++R3) {
                    const long cell = (R1 * n2 + R2) * n3 + R3;
                    const long at = ((long)m * S + mu) * ncell + cell;
                    const double delta = occ ? (double)occ[at] : 1.0;
                    const double lat = (double)imodl(G1 * R1, n1) / n1 + (double)imodl(G2 * R2, n2) / n2
                                     + (double)imodl(G3 * R3, n3) / n3;
                    const double ph = TWO_PI * (lat + gr);
                    const double c = cos(ph), s = sin(ph);
                    for (int k = 0; k < 3; ++k) {
                        const double w = b[mu] * delta * (double)spin[3 * at + k];
                        acc[k][0] += w * c;
                        acc[k][1] += w * s;
                    }
                }
                double* o = F + 2 * 3 * (((int64_t)m * nG + gi) * S + mu);
                for (int k = 0; k < 3; ++k) { o[2 * k] = acc[k][0]; o[2 * k + 1] = acc[k][1]; }
            }
        }
    }
    return 0;
}

/* Debye-Waller factor of one site (Sec. III.A, Eq. dw):
 *   T_mu(G) = (1/(n1 n2 n3)) sum_R < (1 + a_{R,mu}) e^{i G.u_{R,mu}} >
 * with 1 + a = delta / c_mu, c_mu the mean occupancy of the site over every cell
 * and configuration, and < > the mean over configurations; written out that is
 *   T_mu(G) = sum_{m,R} delta e^{2 pi i g.u} / sum_{m,R} delta,
 * a plain average over the occupied atoms of the site.  exact mode (order < 0)
 * evaluates the exponential; order-N mode its Taylor polynomial
 * sum_{k<=N} (i x)^k / k!, x = 2 pi g.u (Sec. III.C, Eq. disp_expansion).
 * A site with no occupied atom gets T = 0.
 * occ [M][S][n1][n2][n3] or NULL (= 1); disp [M][S][n1][n2][n3][3] fractional;
 * T [nG][S][2] output (re, im). */
int orc_dw_mean(const int32_t* n, int32_t S, int32_t M, const float* occ, const float* disp,
                int32_t order, int64_t nG, const int32_t* G, double* T)
{
    if (bad_dims(n) || S < 1 || M < 1 || nG < 0 || !disp || !G || !T) return -1;
    const long ncell = (long)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t gi = 0; gi < nG; ++gi) {
        const double g[3] = {(double)G[3 * gi] / n[0], (double)G[3 * gi + 1] / n[1], (double)G[3 * gi + 2] / n[2]};
        for (int32_t mu = 0; mu < S; ++mu) {
            double tr = 0.0, ti = 0.0, wsum = 0.0;
            for (int32_t m = 0; m < M; ++m)
                for (long cell = 0; cell < ncell; ++cell) {
                    const long at = ((long)m * S + mu) * ncell + cell;
                    const double delta = occ ? (double)occ[at] : 1.0;
                    if (delta == 0.0) continue;
                    const float* u = disp + 3 * at;
                    const double x = TWO_PI * (g[0] * u[0] + g[1] * u[1] + g[2] * u[2]);
                    double er, ei;
                    if (order < 0) {
                        er = cos(x); ei = sin(x);
                    } else {
                        double pr = 1.0, pi = 0.0;      /* (i x)^k / k! */
                        er = 0.0; ei = 0.0;
                        for (int k = 0; k <= order; ++k) {
                            er += pr; ei += pi;
                            const double nr = -pi * x / (k + 1), ni = pr * x / (k + 1);
                            pr = nr; pi = ni;
                        }
                    }
                    tr += delta * er;
                    ti += delta * ei;
                    wsum += delta;
                }
            double* o = T + 2 * (gi * S + mu);
            o[0] = wsum != 0.0 ? tr / wsum : 0.0;
            o[1] = wsum != 0.0 ? ti / wsum : 0.0;
        }
    }
    return 0;
}

/* Method of sub-boxes (Sec. V.A): every lattice point R0 of the supercell is the origin
 * of a sub-box of nsb[0] x nsb[1] x nsb[2] unit cells with open boundaries (its cells
 * R0 + d, 0 <= d_a < nsb_a, taken from the periodic supercell, their positions
 * R0 + d + r_mu + u not folded back), and
 *   F_sb(Q) = sum_{d, mu} b_mu delta e^{2 pi i Q.(d + r_mu + u)}
 * at arbitrary Q (reciprocal-lattice units: Q.x = sum_a Q_a x_a for x in unit-cell
 * coordinates; the common phase e^{2 pi i Q.R0} drops out of |F|^2 and is left out).
 * Outputs, averaged over every origin and configuration:
 *   sq[nQ]        < |F_sb(Q)|^2 >
 *   mean[nQ][2]   < F_sb(Q) >
 * exact mode (order < 0) or the order-N Taylor polynomial of e^{2 pi i Q.u}.
 * occ/disp as orc_sf_nuclear; nsb_a in [1, n_a]. */
int orc_subbox(const int32_t* n, int32_t S, const double* frac, const double* b, int32_t M,
               const float* occ, const float* disp, int32_t order, const int32_t* nsb,
               int64_t nQ, const double* Q, double* sq, double* mean)
{
    if (bad_dims(n) || S < 1 || M < 1 || nQ < 0 || !frac || !b || !nsb || !Q || !sq || !mean) return -1;
    for (int a = 0; a < 3; ++a)
        if (nsb[a] < 1 || nsb[a] > n[a]) return -1;
    const long n1 = n[0], n2 = n[1], n3 = n[2];
    const long ncell = n1 * n2 * n3;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nQ; ++qi) {
        const double* q = Q + 3 * qi;
        double acc_sq = 0.0, acc_r = 0.0, acc_i = 0.0;
        for (int32_t m = 0; m < M; ++m)
        for (long R1 = 0; R1 < n1; ++R1)
        for (long R2 = 0; R2 < n2; ++R2)
        for (long R3 = 0; R3 < n3; ++R3) {
            double fr = 0.0, fi = 0.0;
            for (int32_t mu = 0; mu < S; ++mu)
            for (long d1 = 0; d1 < nsb[0]; ++d1)
            for (long d2 = 0; d2 < nsb[1]; ++d2)
            for (long d3 = 0; d3 < nsb[2]; ++d3) {
                const long cell = (((R1 + d1) % n1) * n2 + (R2 + d2) % n2) * n3 + (R3 + d3) % n3;
                const long at = ((long)m * S + mu) * ncell + cell;
                const double delta = occ ? (double)occ[at] : 1.0;
                if (delta == 0.0) continue;
                const double x = q[0] * (d1 + frac[3 * mu]) + q[1] * (d2 + frac[3 * mu + 1]) +
                                 q[2] * (d3 + frac[3 * mu + 2]);
                double gu = 0.0;
                if (disp) {
                    const float* u = disp + 3 * at;
                    gu = q[0] * u[0] + q[1] * u[1] + q[2] * u[2];
                }
                double er, ei;
                if (order < 0) {
                    er = cos(TWO_PI * (x + gu)); ei = sin(TWO_PI * (x + gu));
                } else {
                    const double c = cos(TWO_PI * x), s = sin(TWO_PI * x), y = TWO_PI * gu;
                    double pr = 1.0, pi = 0.0, tr = 0.0, ti = 0.0;
                    for (int k = 0; k <= order; ++k) {
                        tr += pr; ti += pi;
                        const double nr = -pi * y / (k + 1), ni = pr * y / (k + 1);
                        pr = nr; pi = ni;
                    }
                    er = c * tr - s * ti; ei = c * ti + s * tr;
                }
                fr += b[mu] * delta * er;
                fi += b[mu] * delta * ei;
            }
            acc_sq += fr * fr + fi * fi;
            acc_r += fr;
            acc_i += fi;
        }
        const double cnt = (double)M * ncell;
        sq[qi] = acc_sq / cnt;
        mean[2 * qi] = acc_r / cnt;
        mean[2 * qi + 1] = acc_i / cnt;
    }
    return 0;
}

/* Pair double sum for ONE configuration at integer supercell points G:
 *   out(G) = (1/normN) sum_{j,k} b_j d_j b_k d_k e^{2 pi i g.(x_j - x_k)}
 * where x = R + r_mu + u in unit-cell coordinates and each separation is mapped to
 * its nearest image: (x_j - x_k)_a / n_a brought into [-1/2, 1/2) (Sec. II).
 * out [nG][2]. */
int orc_pair_sum(const int32_t* n, int32_t S, const double* frac, const double* b,
                 const float* occ, const float* disp, double normN,
                 int64_t nG, const int32_t* G, double* out)
{
    if (bad_dims(n) || S < 1 || nG < 0 || !frac || !b || !G || !out || !(normN > 0)) return -1;
    const long n1 = n[0], n2 = n[1], n3 = n[2];
    const long ncell = n1 * n2 * n3;
    const long natom = ncell * S;
    const double nd[3] = {(double)n1, (double)n2, (double)n3};
    double* pos = (double*)malloc(sizeof(double) * 3 * natom);
    double* w = (double*)malloc(sizeof(double) * natom);
    if (!pos || !w) { free(pos); free(w); return -1; }
    for (int32_t mu = 0; mu < S; ++mu)
        for (long R1 = 0; R1 < n1; ++R1)
        for (long R2 = 0; R2 < n2; ++R2)
        for (long R3 = 0; R3 < n3; ++R3) {
            const long cell = (R1 * n2 + R2) * n3 + R3;
            const long at = (long)mu * ncell + cell;
            const double R[3] = {(double)R1, (double)R2, (double)R3};
            for (int a = 0; a < 3; ++a)
                pos[3 * at + a] = R[a] + frac[3 * mu + a] + (disp ? (double)disp[3 * at + a] : 0.0);
            w[at] = b[mu] * (occ ? (double)occ[at] : 1.0);
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t gi = 0; gi < nG; ++gi) {
        const double Gv[3] = {(double)G[3 * gi], (double)G[3 * gi + 1], (double)G[3 * gi + 2]};
        double sr = 0.0, si = 0.0;
        for (long j = 0; j < natom; ++j) {
            if (w[j] == 0.0) continue;
            for (long k = 0; k < natom; ++k) {
                if (w[k] == 0.0) continue;
                double ph = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double d = (pos[3 * j + a] - pos[3 * k + a]) / nd[a];   /* supercell fraction */
                    d -= floor(d + 0.5);                                     /* nearest image */
                    ph += Gv[a] * d;                                         /* g_a * d n_a = G_a d */
                }
                ph *= TWO_PI;
                sr += w[j] * w[k] * cos(ph);
                si += w[j] * w[k] * sin(ph);
            }
        }
        out[2 * gi] = sr / normN;
        out[2 * gi + 1] = si / normN;
    }
    free(pos); free(w);
    return 0;
}

static double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

/* One-axis factor of the windowed-sinc weight W = W_sinc * L:
 * 2 r_cut sinc(2 pi r_cut d) * [ |d| < w ] sinc(pi d / w).  The plain filter has
 * r_cut = (1 - 1/m)/2 and w = m; the m' modification takes r_cut = (1 - 1/m)/m' and
 * replaces m by w = m m'/2 in the window, so that m' = 2 is the plain filter. */
static double lanczos_axis(double d, int m, int mp)
{
    const double rcut = (1.0 - 1.0 / m) / mp;
    const double w = 0.5 * m * mp;
    if (!(fabs(d) < w)) return 0.0;
    return 2.0 * rcut * sinc(TWO_PI * rcut * d) * sinc(M_PI * d / w);
}

/* Windowed sum at one Q: G_a in [floor(Q_a) - w + 1, floor(Q_a) + w] with w = m m'/2.
 * Returns -1 if a needed G lies outside the input box. */
static int lanczos_at(const double* Q, int m, int mp, const int32_t* e0, const int32_t* ecount,
                      const double* I, double* out)
{
    const long w = (long)m * mp / 2;
    const long f[3] = {(long)floor(Q[0]), (long)floor(Q[1]), (long)floor(Q[2])};
    double num = 0.0, den = 0.0;
    for (long G1 = f[0] - w + 1; G1 <= f[0] + w; ++G1)
    for (long G2 = f[1] - w + 1; G2 <= f[1] + w; ++G2)
    for (long G3 = f[2] - w + 1; G3 <= f[2] + w; ++G3) {
        const long j1 = G1 - e0[0], j2 = G2 - e0[1], j3 = G3 - e0[2];
        if (j1 < 0 || j2 < 0 || j3 < 0 || j1 >= ecount[0] || j2 >= ecount[1] || j3 >= ecount[2]) return -1;
        const double W = lanczos_axis(Q[0] - G1, m, mp) * lanczos_axis(Q[1] - G2, m, mp) *
                         lanczos_axis(Q[2] - G3, m, mp);
        num += W * I[(j1 * ecount[1] + j2) * ecount[2] + j3];
        den += W;
    }
    *out = num / den;
    return 0;
}

/* Windowed-sinc resampling, direct (2w)^3 sum, w = m m'/2 (mp = m' >= 2, m m' even).
 * Input I(G) on the box [e0, e0 + ecount) (last axis fastest).
 * Output I(Q) at Q_a = q0_a + i_a / s for i_a in [0, qcount_a) (last axis fastest):
 *   I(Q) = sum_G I(G) W(Q - G) / sum_G W(Q - G),
 *   G_a in [floor(Q_a) - w + 1, floor(Q_a) + w].
 * Returns -1 if a needed G lies outside the input box. */
int orc_lanczos_cutoff(int32_t m, int32_t mp, int32_t s, const int32_t* e0, const int32_t* ecount,
                       const double* I, const int32_t* q0, const int32_t* qcount, double* out)
{
    if (m < 2 || mp < 2 || (m * mp) % 2 != 0 || s < 1 || !e0 || !ecount || !I || !q0 || !qcount || !out)
        return -1;
    const long w = (long)m * mp / 2;
    /* range check over the whole output first */
    for (int a = 0; a < 3; ++a) {
        const long lo = (long)q0[a] - w + 1;
        const long hi = (long)q0[a] + (qcount[a] - 1) / s + w;
        if (lo < e0[a] || hi >= (long)e0[a] + ecount[a]) return -1;
    }
    const long total = (long)qcount[0] * qcount[1] * qcount[2];
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|:bad)
    for (long idx = 0; idx < total; ++idx) {
        const long i3 = idx % qcount[2], i2 = (idx / qcount[2]) % qcount[1], i1 = idx / ((long)qcount[2] * qcount[1]);
        const double Q[3] = {q0[0] + (double)i1 / s, q0[1] + (double)i2 / s, q0[2] + (double)i3 / s};
        if (lanczos_at(Q, m, mp, e0, ecount, I, &out[idx]) != 0) bad = 1;
    }
    return bad ? -1 : 0;
}

int orc_lanczos(int32_t m, int32_t s, const int32_t* e0, const int32_t* ecount, const double* I,
                const int32_t* q0, const int32_t* qcount, double* out)
{
    return orc_lanczos_cutoff(m, 2, s, e0, ecount, I, q0, qcount, out);
}

/* The same windowed sum at npts arbitrary points Q[npts][3] (reciprocal-lattice
 * units, any direction, e.g. an off-axis plane).  Returns -1 if a needed G lies
 * outside the input box. */
int orc_lanczos_points(int32_t m, int32_t mp, const int32_t* e0, const int32_t* ecount, const double* I,
                       int64_t npts, const double* Q, double* out)
{
    if (m < 2 || mp < 2 || (m * mp) % 2 != 0 || npts < 0 || !e0 || !ecount || !I || !Q || !out) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|:bad)
    for (int64_t i = 0; i < npts; ++i)
        if (lanczos_at(Q + 3 * i, m, mp, e0, ecount, I, &out[i]) != 0) bad = 1;
    return bad ? -1 : 0;
}

/* x^-3 (sin x - x cos x) = sin(x)/x^3 - cos(x)/x^2: the bracket of W_r (the Fourier
 * transform of a ball of radius 1 divided by 4 pi).  Near 0 its series
 * 1/3 - x^2/30 + x^4/840 avoids the cancellation. */
double orc_ball_ft(double x)
{
    const double ax = fabs(x);
    if (ax < 1e-2) return 1.0 / 3.0 - x * x / 30.0 + x * x * x * x / 840.0;
    return (sin(ax) - ax * cos(ax)) / (ax * ax * ax);
}

/* Lanczos resampling with the spherical cutoff (Sec. V.B, the third modification):
 * W = W_r(|Q - G|) * L(Q - G), W_r proportional to orc_ball_ft(|Q - G|_cart r_c)
 * with r_c = (1 - 1/m) r_max, L the window of Eq. lanczos (unchanged, half-width m).
 * recip[9] = rows a*, b*, c* (inverse Angstrom, 2 pi included); n[3] the supercell;
 * Q - G in supercell-grid units is (Q_a - G_a)/n_a reciprocal-lattice units.
 * Box and output conventions as orc_lanczos_cutoff (m' = 2).  The constant factor
 * 4 pi r_c^3 / (n1 n2 n3 V) cancels in the normalised sum. */
int orc_lanczos_spherical(int32_t m, int32_t s, const int32_t* e0, const int32_t* ecount, const double* I,
                          const int32_t* q0, const int32_t* qcount, const double* recip, const int32_t* n,
                          double rc, double* out)
{
    if (m < 2 || s < 1 || !e0 || !ecount || !I || !q0 || !qcount || !recip || !n || !out || !(rc > 0.0)) return -1;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1) return -1;
        const long lo = (long)q0[a] - m + 1;
        const long hi = (long)q0[a] + (qcount[a] - 1) / s + m;
        if (lo < e0[a] || hi >= (long)e0[a] + ecount[a]) return -1;
    }
    const long total = (long)qcount[0] * qcount[1] * qcount[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (long idx = 0; idx < total; ++idx) {
        const long i3 = idx % qcount[2], i2 = (idx / qcount[2]) % qcount[1], i1 = idx / ((long)qcount[2] * qcount[1]);
        const double Q[3] = {q0[0] + (double)i1 / s, q0[1] + (double)i2 / s, q0[2] + (double)i3 / s};
        const long f[3] = {(long)floor(Q[0]), (long)floor(Q[1]), (long)floor(Q[2])};
        double num = 0.0, den = 0.0;
        for (long G1 = f[0] - m + 1; G1 <= f[0] + m; ++G1)
        for (long G2 = f[1] - m + 1; G2 <= f[1] + m; ++G2)
        for (long G3 = f[2] - m + 1; G3 <= f[2] + m; ++G3) {
            const double d[3] = {Q[0] - G1, Q[1] - G2, Q[2] - G3};
            double L = 1.0;
            for (int a = 0; a < 3; ++a) L *= fabs(d[a]) < m ? sinc(M_PI * d[a] / m) : 0.0;
            double q[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) q[c] += d[a] / n[a] * recip[3 * a + c];
            const double W = orc_ball_ft(sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) * rc) * L;
            const long j1 = G1 - e0[0], j2 = G2 - e0[1], j3 = G3 - e0[2];
            num += W * I[(j1 * ecount[1] + j2) * ecount[2] + j3];
            den += W;
        }
        out[idx] = num / den;
    }
    return 0;
}

int orc_version(void) { return 1; }
