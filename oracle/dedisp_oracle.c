/*
 * CPU oracle for the direct incoherent dedispersion transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the GPU library: every number below is derived here from the paper
 * (Barsdell, Bailes, Barnes & Fluke 2012, "Accelerating incoherent
 * dedispersion", MNRAS 422, 379).
 *
 * It is deliberately plain and slow: each output is the sum of the definition
 * written out, one channel at a time, decoding every sample from the packed
 * input at the moment it is used.  Parallelism over DM rows (OpenMP) changes
 * no arithmetic: every output is an independent integer sum.
 *
 * Readings of the paper that this file fixes (listed in the design notes):
 *   - channel c is at frequency f_top + c*df (f_top = start of the band),
 *   - "rounded to the nearest integer" is round-half-away-from-zero,
 *   - the delay is evaluated in IEEE binary64 in the order written below,
 *   - outputs exist for 0 <= t < nsamps - max_delay only,
 *   - samples are raw unsigned codes; 2-bit samples are packed four per byte,
 *     channel c at bits [2*(c%4), 2*(c%4)+1] of byte c/4 of its time row.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Dispersion constant k_DM in MHz^2 pc^-1 cm^3 s (Section 1, the dispersion
 * delay equation).  The paper notes the common 1/2.41e-4 approximation and
 * gives this value as the constant itself. */
static const double ORACLE_K_DM = 4.148808e3;

enum {
    ORACLE_OK = 0,
    ORACLE_BAD_ARG = -1,
    ORACLE_TOO_FEW_SAMPLES = -2
};

/* Same acceptance rules as the library's public interface: the transform is
 * only defined here for a band that descends from f_top (df < 0) and stays
 * at positive frequency, 2- or 8-bit codes, whole bytes per time row. */
static int oracle_check_params(int nchans, double dt, double f_top, double df, int nbits)
{
    if (nchans <= 0) return ORACLE_BAD_ARG;
    if (nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    if (((long long)nchans * nbits) % 8 != 0) return ORACLE_BAD_ARG;
    if (!(dt > 0.0) || !isfinite(dt)) return ORACLE_BAD_ARG;
    if (!(f_top > 0.0) || !isfinite(f_top)) return ORACLE_BAD_ARG;
    if (!(df < 0.0) || !isfinite(df)) return ORACLE_BAD_ARG;
    if (!(f_top + (double)(nchans - 1) * df > 0.0)) return ORACLE_BAD_ARG;
    return ORACLE_OK;
}

/* Delta T(nu) of the "partial_delay" equation of Section 2.1: the delay in
 * samples per unit DM of channel nu relative to the start of the band,
 *   (k_DM / dtau) * ( 1/(nu0 + nu*dnu)^2 - 1/nu0^2 ). */
int oracle_partial_delay(int nchans, double dt, double f_top, double df, double* dT)
{
    if (!dT) return ORACLE_BAD_ARG;
    if (oracle_check_params(nchans, dt, f_top, df, 8) != ORACLE_OK) return ORACLE_BAD_ARG;
    const double inv_top2 = 1.0 / (f_top * f_top);
    const double scale = ORACLE_K_DM / dt;
    for (int nu = 0; nu < nchans; ++nu) {
        const double f = f_top + (double)nu * df;
        dT[nu] = scale * (1.0 / (f * f) - inv_top2);
    }
    return ORACLE_OK;
}

/* Delta t(d, nu) of the "delay" equation of Section 2.1:
 * round(DM(d) * Delta T(nu)), for every trial DM (rows) and channel
 * (columns).  Also returns the largest delay, which fixes how many outputs
 * exist. */
int oracle_delay_table(int nchans, double dt, double f_top, double df,
                       const double* dms, int ndm, int32_t* table, int32_t* max_delay)
{
    if (!dms || !table || !max_delay || ndm <= 0) return ORACLE_BAD_ARG;
    if (oracle_check_params(nchans, dt, f_top, df, 8) != ORACLE_OK) return ORACLE_BAD_ARG;
    for (int d = 0; d < ndm; ++d)
        if (!(dms[d] >= 0.0) || !isfinite(dms[d])) return ORACLE_BAD_ARG;

    const double inv_top2 = 1.0 / (f_top * f_top);
    const double scale = ORACLE_K_DM / dt;
    int32_t mx = 0;
    for (int d = 0; d < ndm; ++d) {
        for (int nu = 0; nu < nchans; ++nu) {
            const double f = f_top + (double)nu * df;
            const double dTnu = scale * (1.0 / (f * f) - inv_top2);
            const double v = round(dms[d] * dTnu);      /* half away from zero */
            if (!(v < 2147483647.0)) return ORACLE_BAD_ARG;
            const int32_t di = (int32_t)v;
            table[(size_t)d * nchans + nu] = di;
            if (di > mx) mx = di;
        }
    }
    *max_delay = mx;
    return ORACLE_OK;
}

/* A[nu][t]: the unsigned code of channel nu at time sample t, read straight
 * from the packed time-major input. */
static inline uint32_t oracle_sample(const uint8_t* in, int nchans, int nbits,
                                     int64_t t, int nu)
{
    if (nbits == 8)
        return in[(size_t)t * (size_t)nchans + (size_t)nu];
    const size_t row_bytes = (size_t)nchans / 4;
    const uint8_t byte = in[(size_t)t * row_bytes + (size_t)(nu / 4)];
    return (uint32_t)((byte >> (2 * (nu % 4))) & 3u);
}

/* The direct dedispersion transform, the "direct" equation of Section 2.1:
 *   D[d][t] = sum over nu = 0..N_nu-1 of A[nu][t + Delta t(d, nu)]
 * for 0 <= d < ndm and 0 <= t < nsamps - max_delay, written to
 * out[d * out_stride + t].
 * With a channel kill mask (Section 2.3; NULL = every channel on), each
 * term is multiplied by mask[nu] in {0, 1}, the arithmetic form of the mask
 * the paper describes; the delays and the output range are unchanged. */
int oracle_dedisperse(const uint8_t* in, int64_t nsamps, int nchans, int nbits,
                      const int32_t* table, int ndm, int32_t max_delay,
                      uint32_t* out, int64_t out_stride, int nthreads, const int32_t* mask)
{
    if (!in || !table || !out || ndm <= 0 || nchans <= 0) return ORACLE_BAD_ARG;
    if (nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    if (nbits == 2 && nchans % 4) return ORACLE_BAD_ARG;
    if (nsamps <= (int64_t)max_delay) return ORACLE_TOO_FEW_SAMPLES;
    const int64_t nout = nsamps - (int64_t)max_delay;
    if (out_stride < nout) return ORACLE_BAD_ARG;
    for (size_t i = 0; i < (size_t)ndm * (size_t)nchans; ++i)
        if (table[i] < 0 || table[i] > max_delay) return ORACLE_BAD_ARG;
    if (mask)
        for (int nu = 0; nu < nchans; ++nu)
            if (mask[nu] != 0 && mask[nu] != 1) return ORACLE_BAD_ARG;

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int d = 0; d < ndm; ++d) {
        const int32_t* delay = table + (size_t)d * nchans;
        uint32_t* row = out + (size_t)d * (size_t)out_stride;
        for (int64_t t = 0; t < nout; ++t) {
            uint32_t sum = 0;
            for (int nu = 0; nu < nchans; ++nu)
                sum += (mask ? (uint32_t)mask[nu] : 1u) *
                       oracle_sample(in, nchans, nbits, t + delay[nu], nu);
            row[t] = sum;
        }
    }
    return ORACLE_OK;
}

/* The same definition evaluated only at the listed (d, t) points, for
 * checking sampled outputs of inputs too large to transform whole on a CPU. */
int oracle_dedisperse_points(const uint8_t* in, int64_t nsamps, int nchans, int nbits,
                             const int32_t* table, int ndm, int32_t max_delay,
                             const int64_t* d_idx, const int64_t* t_idx, int64_t npts,
                             uint32_t* out, int nthreads, const int32_t* mask)
{
    if (!in || !table || !out || !d_idx || !t_idx || npts < 0) return ORACLE_BAD_ARG;
    if (nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    if (nbits == 2 && nchans % 4) return ORACLE_BAD_ARG;
    if (nsamps <= (int64_t)max_delay) return ORACLE_TOO_FEW_SAMPLES;
    const int64_t nout = nsamps - (int64_t)max_delay;
    for (int64_t i = 0; i < npts; ++i)
        if (d_idx[i] < 0 || d_idx[i] >= ndm || t_idx[i] < 0 || t_idx[i] >= nout)
            return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        const int32_t* delay = table + (size_t)d_idx[i] * nchans;
        const int64_t t = t_idx[i];
        uint32_t sum = 0;
        for (int nu = 0; nu < nchans; ++nu)
            sum += (mask ? (uint32_t)mask[nu] : 1u) *
                   oracle_sample(in, nchans, nbits, t + delay[nu], nu);
        out[i] = sum;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Time-scrunching (Section 2.1).  Beyond the "diagonal" DM -- where the
 * dispersion trail crosses more than one time sample per frequency channel
 * -- the time resolution is halved by adding adjacent pairs of samples, and
 * halved again at twice that DM, and so on.  The trials of a scrunched group
 * are then dedispersed with the same direct sum at the coarser resolution.
 *
 * Readings fixed here:
 *   - the diagonal DM is the DM at which the delay between the last two
 *     channels of the band (where the trail is steepest) is one sample:
 *     1 / (Delta T(N-1) - Delta T(N-2));
 *   - a trial scrunches by 2 once its DM exceeds the diagonal, by 4 once it
 *     exceeds twice the diagonal, and so on (up to a caller-given maximum);
 *   - a group with factor s uses the delay equation with the sampling time
 *     s*dtau, scrunched sample t' is the sum of samples s*t' .. s*t'+s-1
 *     (a trailing partial group of fewer than s samples is dropped), and the
 *     group's outputs exist for t' < nsamps/s - (largest delay of the group).
 * ------------------------------------------------------------------------ */

/* The diagonal DM of the band. */
int oracle_diagonal_dm(int nchans, double dt, double f_top, double df, double* dm)
{
    if (!dm) return ORACLE_BAD_ARG;
    if (oracle_check_params(nchans, dt, f_top, df, 8) != ORACLE_OK) return ORACLE_BAD_ARG;
    if (nchans < 2) {
        *dm = HUGE_VAL;             /* one channel: no trail to smear */
        return ORACLE_OK;
    }
    const double inv_top2 = 1.0 / (f_top * f_top);
    const double scale = ORACLE_K_DM / dt;
    const double fa = f_top + (double)(nchans - 2) * df;
    const double fb = f_top + (double)(nchans - 1) * df;
    const double dTa = scale * (1.0 / (fa * fa) - inv_top2);
    const double dTb = scale * (1.0 / (fb * fb) - inv_top2);
    *dm = 1.0 / (dTb - dTa);
    return ORACLE_OK;
}

/* The scrunch factor of one trial DM: 1 up to the diagonal, then doubling
 * each time the DM exceeds the next power-of-two multiple of it. */
int oracle_scrunch_factor(double dm, double dm_diag, int max_factor)
{
    int s = 1;
    double threshold = dm_diag;
    while (s < max_factor && dm > threshold) {
        s *= 2;
        threshold *= 2.0;
    }
    return s;
}

/* x[t'][c] = sum over i < s of A[c][s*t' + i], for t' < nsamps / s, as
 * unpacked time-major uint32 values. */
int oracle_scrunch(const uint8_t* in, int64_t nsamps, int nchans, int nbits, int s,
                   uint32_t* out)
{
    if (!in || !out || nsamps < 0 || s < 1) return ORACLE_BAD_ARG;
    if (nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    if (nbits == 2 && nchans % 4) return ORACLE_BAD_ARG;
    const int64_t n = nsamps / s;
    for (int64_t tp = 0; tp < n; ++tp)
        for (int nu = 0; nu < nchans; ++nu) {
            uint32_t sum = 0;
            for (int i = 0; i < s; ++i)
                sum += oracle_sample(in, nchans, nbits, tp * s + i, nu);
            out[(size_t)tp * (size_t)nchans + (size_t)nu] = sum;
        }
    return ORACLE_OK;
}

/* The direct transform (the "direct" equation of Section 2.1) of unpacked
 * time-major values x[t][c] (such as scrunched samples), with an optional
 * 0/1 channel kill mask, for 0 <= t < nsamps - max_delay. */
int oracle_dedisperse_values(const uint32_t* x, int64_t nsamps, int nchans,
                             const int32_t* table, int ndm, int32_t max_delay,
                             uint32_t* out, int64_t out_stride, int nthreads,
                             const int32_t* mask)
{
    if (!x || !table || !out || ndm <= 0 || nchans <= 0) return ORACLE_BAD_ARG;
    if (nsamps <= (int64_t)max_delay) return ORACLE_TOO_FEW_SAMPLES;
    const int64_t nout = nsamps - (int64_t)max_delay;
    if (out_stride < nout) return ORACLE_BAD_ARG;
    for (size_t i = 0; i < (size_t)ndm * (size_t)nchans; ++i)
        if (table[i] < 0 || table[i] > max_delay) return ORACLE_BAD_ARG;
    if (mask)
        for (int nu = 0; nu < nchans; ++nu)
            if (mask[nu] != 0 && mask[nu] != 1) return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int d = 0; d < ndm; ++d) {
        const int32_t* delay = table + (size_t)d * nchans;
        uint32_t* row = out + (size_t)d * (size_t)out_stride;
        for (int64_t t = 0; t < nout; ++t) {
            uint32_t sum = 0;
            for (int nu = 0; nu < nchans; ++nu)
                sum += (mask ? (uint32_t)mask[nu] : 1u) *
                       x[(size_t)(t + delay[nu]) * (size_t)nchans + (size_t)nu];
            row[t] = sum;
        }
    }
    return ORACLE_OK;
}

/* The scrunched transform of one factor group at the listed (d, t') points:
 * sum over channels of the s input samples that make up scrunched sample
 * t' + delay[d][c], table being the group's delay table at s times the
 * sampling time.  For checking sampled outputs of inputs too large to
 * transform whole on a CPU. */
int oracle_dedisperse_scrunched_points(const uint8_t* in, int64_t nsamps, int nchans, int nbits,
                                       int s, const int32_t* table, int ndm, int32_t max_delay,
                                       const int64_t* d_idx, const int64_t* t_idx, int64_t npts,
                                       uint32_t* out, int nthreads, const int32_t* mask)
{
    if (!in || !table || !out || !d_idx || !t_idx || npts < 0 || s < 1) return ORACLE_BAD_ARG;
    if (nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    if (nbits == 2 && nchans % 4) return ORACLE_BAD_ARG;
    const int64_t n = nsamps / s;
    if (n <= (int64_t)max_delay) return ORACLE_TOO_FEW_SAMPLES;
    const int64_t nout = n - (int64_t)max_delay;
    for (int64_t i = 0; i < npts; ++i)
        if (d_idx[i] < 0 || d_idx[i] >= ndm || t_idx[i] < 0 || t_idx[i] >= nout)
            return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        const int32_t* delay = table + (size_t)d_idx[i] * nchans;
        uint32_t sum = 0;
        for (int nu = 0; nu < nchans; ++nu) {
            const int64_t t0 = (t_idx[i] + delay[nu]) * s;
            uint32_t v = 0;
            for (int j = 0; j < s; ++j) v += oracle_sample(in, nchans, nbits, t0 + j, nu);
            sum += (mask ? (uint32_t)mask[nu] : 1u) * v;
        }
        out[i] = sum;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Sub-band dedispersion (Section 4, with the sub-bands aligned on their
 * early edge as Appendix B assumes).  The nchans channels form nsb = nchans /
 * nsub sub-bands of nsub channels, sub-band n starting at channel n*nsub.
 * The trials form groups of ngroup consecutive list entries; the group's
 * first trial is its nominal DM.
 *
 * Step 1 dedisperses each sub-band at every nominal DM, relative to the
 * sub-band's first channel:
 *   S[n][m][t] = sum over j < nsub of A[n*nsub + j][t + dt(m, n*nsub + j) - dt(m, n*nsub)]
 * for t < len1 = nsamps - (largest such relative delay over n, m, j).
 * Step 2 dedisperses, for every trial d of nominal m = d / ngroup, the
 * "miniature filterbank" of the nsb sub-band series of m with the trial's
 * delay at each sub-band's first channel:
 *   D[d][t] = sum over n of S[n][m][t + dt(d, n*nsub)]
 * for t < nout = len1 - (largest dt(d, n*nsub)).
 * dt(m, c) are rows of the delay table at the nominal DMs (tab_nom, [nnom]
 * rows), dt(d, c) rows of the trials' table (tab, [ndm] rows).
 * ------------------------------------------------------------------------ */

/* len1 and nout of the two-step definition above. */
int oracle_subband_lengths(int64_t nsamps, int nchans, int nsub, const int32_t* tab_nom,
                           int nnom, const int32_t* tab, int ndm, int64_t* len1, int64_t* nout)
{
    if (!tab_nom || !tab || !len1 || !nout || nsub <= 0 || nchans % nsub) return ORACLE_BAD_ARG;
    int32_t mx1 = 0, mx2 = 0;
    for (int m = 0; m < nnom; ++m)
        for (int c = 0; c < nchans; ++c) {
            const int32_t r = tab_nom[(size_t)m * nchans + c] - tab_nom[(size_t)m * nchans + (c / nsub) * nsub];
            if (r < 0) return ORACLE_BAD_ARG;
            if (r > mx1) mx1 = r;
        }
    for (int d = 0; d < ndm; ++d)
        for (int n = 0; n < nchans / nsub; ++n) {
            const int32_t v = tab[(size_t)d * nchans + n * nsub];
            if (v < 0) return ORACLE_BAD_ARG;
            if (v > mx2) mx2 = v;
        }
    *len1 = nsamps - mx1;
    *nout = *len1 - mx2;
    return (*len1 > 0 && *nout > 0) ? ORACLE_OK : ORACLE_TOO_FEW_SAMPLES;
}

/* Step 1: S [nsb][nnom][len1], with an optional 0/1 channel kill mask. */
int oracle_subband_step1(const uint8_t* in, int64_t nsamps, int nchans, int nbits, int nsub,
                         const int32_t* tab_nom, int nnom, int64_t len1, uint32_t* S,
                         int nthreads, const int32_t* mask)
{
    if (!in || !tab_nom || !S || nsub <= 0 || nchans % nsub || nnom <= 0 || len1 <= 0)
        return ORACLE_BAD_ARG;
    if (nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    const int nsb = nchans / nsub;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int n = 0; n < nsb; ++n)
        for (int m = 0; m < nnom; ++m) {
            const int32_t* dl = tab_nom + (size_t)m * nchans;
            const int c0 = n * nsub;
            uint32_t* row = S + ((size_t)n * nnom + m) * (size_t)len1;
            for (int64_t t = 0; t < len1; ++t) {
                uint32_t sum = 0;
                for (int j = 0; j < nsub; ++j) {
                    const int c = c0 + j;
                    const int64_t ts = t + dl[c] - dl[c0];
                    if (ts >= nsamps) continue;           /* not reached for t < len1 */
                    sum += (mask ? (uint32_t)mask[c] : 1u) * oracle_sample(in, nchans, nbits, ts, c);
                }
                row[t] = sum;
            }
        }
    return ORACLE_OK;
}

/* Step 2: D [ndm][out_stride], t < nout. */
int oracle_subband_step2(const uint32_t* S, int nsb, int nnom, int64_t len1, int nchans, int nsub,
                         const int32_t* tab, int ndm, int ngroup, int64_t nout, uint32_t* out,
                         int64_t out_stride, int nthreads)
{
    if (!S || !tab || !out || nsub <= 0 || nsb * nsub != nchans || ngroup <= 0) return ORACLE_BAD_ARG;
    if ((ndm + ngroup - 1) / ngroup > nnom || out_stride < nout) return ORACLE_BAD_ARG;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int d = 0; d < ndm; ++d) {
        const int m = d / ngroup;
        const int32_t* dl = tab + (size_t)d * nchans;
        uint32_t* row = out + (size_t)d * (size_t)out_stride;
        for (int64_t t = 0; t < nout; ++t) {
            uint32_t sum = 0;
            for (int n = 0; n < nsb; ++n)
                sum += S[((size_t)n * nnom + m) * (size_t)len1 + (size_t)(t + dl[n * nsub])];
            row[t] = sum;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Tree dedispersion (Section 3).  Step i (radix r = 2^i) builds, out of
 * place, A^{i+1}[2v][t]   = A^i[Phi(r, 2v)][t] + A^i[Phi(r, 2v+1)][t + Theta(i, 2v)]
 *            A^{i+1}[2v+1][t] = A^i[Phi(r, 2v)][t] + A^i[Phi(r, 2v+1)][t + Theta(i, 2v+1)]
 * with the delay function Theta(i, v) = ((v mod 2^{i+1}) + 1) / 2 and the
 * shuffle Phi(r, v) = (v mod 2) r + v/2 + (v/(2r)) r, divisions truncating.
 * After k steps, rows b*2^k + d' (d' < 2^k) hold the tree transform of the
 * block of 2^k channels starting at b*2^k at tree DM d'.  Reading fixed here:
 * a step is defined where every sample it reads exists, so A^{i+1} has 2^i
 * fewer samples than A^i and k steps leave nsamps - (2^k - 1).
 * ------------------------------------------------------------------------ */

static int oracle_tree_theta(int i, int v) { return ((v % (1 << (i + 1))) + 1) / 2; }

static int oracle_tree_phi(int r, int v) { return (v % 2) * r + v / 2 + (v / (2 * r)) * r; }

/* k steps of the tree over every channel (nchans a multiple of 2^k), with an
 * optional 0/1 kill mask applied to the input: out [nchans][nsamps - (2^k - 1)]. */
/* The k tree steps on the channel-major input -- packed codes `in` of nbits
 * bits, or (in = NULL) unpacked time-major values `vals` [nsamps][nchans] --
 * with channel v read slope * (v mod 2^k) samples later (slope = 0: the input
 * as it is). */
static int tree_steps(const uint8_t* in, const uint32_t* vals, int64_t nsamps, int nchans, int nbits,
                      int k, int slope, uint32_t* out, const int32_t* mask)
{
    if ((!in && !vals) || !out || k < 0 || k > 20 || nchans <= 0 || nchans % (1 << k) || slope < 0)
        return ORACLE_BAD_ARG;
    if (in && nbits != 2 && nbits != 8) return ORACLE_BAD_ARG;
    const int B = 1 << k;
    const int64_t ns = nsamps - (int64_t)slope * (B - 1);   /* samples every channel has */
    const int64_t n_out = ns - (B - 1);
    if (n_out <= 0) return ORACLE_TOO_FEW_SAMPLES;
    const size_t cells = (size_t)nchans * (size_t)ns;
    uint32_t* a = (uint32_t*)malloc(cells * sizeof(uint32_t));
    uint32_t* b = (uint32_t*)malloc(cells * sizeof(uint32_t));
    if (!a || !b) {
        free(a);
        free(b);
        return ORACLE_BAD_ARG;
    }
    /* A^0 = the input, channel-major, with the imposed delay */
    for (int v = 0; v < nchans; ++v) {
        const int64_t shift = (int64_t)slope * (v % B);
        for (int64_t t = 0; t < ns; ++t) {
            const uint32_t x = in ? oracle_sample(in, nchans, nbits, t + shift, v)
                                  : vals[(size_t)(t + shift) * (size_t)nchans + (size_t)v];
            a[(size_t)v * ns + t] = (mask ? (uint32_t)mask[v] : 1u) * x;
        }
    }
    int64_t len = ns;
    for (int i = 0; i < k; ++i) {
        const int r = 1 << i;
        const int64_t next = len - r;       /* largest Theta(i, .) is 2^i */
        for (int v = 0; v < nchans / 2; ++v) {
            const uint32_t* lo = a + (size_t)oracle_tree_phi(r, 2 * v) * ns;
            const uint32_t* hi = a + (size_t)oracle_tree_phi(r, 2 * v + 1) * ns;
            const int th0 = oracle_tree_theta(i, 2 * v), th1 = oracle_tree_theta(i, 2 * v + 1);
            uint32_t* o0 = b + (size_t)(2 * v) * ns;
            uint32_t* o1 = b + (size_t)(2 * v + 1) * ns;
            for (int64_t t = 0; t < next; ++t) {
                o0[t] = lo[t] + hi[t + th0];
                o1[t] = lo[t] + hi[t + th1];
            }
        }
        uint32_t* tmp = a;
        a = b;
        b = tmp;
        len = next;
    }
    for (int v = 0; v < nchans; ++v)
        for (int64_t t = 0; t < n_out; ++t)
            out[(size_t)v * n_out + t] = a[(size_t)v * ns + t];
    free(a);
    free(b);
    return ORACLE_OK;
}

int oracle_tree(const uint8_t* in, int64_t nsamps, int nchans, int nbits, int k,
                uint32_t* out, const int32_t* mask)
{
    return tree_steps(in, NULL, nsamps, nchans, nbits, k, 0, out, mask);
}

/* Stage 1 for DMs beyond the piecewise diagonal (Section 3, computing larger
 * DMs): a time delay is imposed across each block of 2^k channels before the
 * tree steps -- channel v is read slope * (v mod 2^k) samples later, a
 * diagonal of `slope` samples per channel -- so tree row d' of a block then
 * covers a trail of slope * 2^k + d' samples from the block's first channel
 * to the next block's.  Output [nchans][nsamps - (slope + 1)(2^k - 1)];
 * slope 0 is oracle_tree. */
int oracle_tree_imposed(const uint8_t* in, int64_t nsamps, int nchans, int nbits, int k, int slope,
                        uint32_t* out, const int32_t* mask)
{
    return tree_steps(in, NULL, nsamps, nchans, nbits, k, slope, out, mask);
}

/* The same pass over unpacked time-major values x [nsamps][nchans] (such as
 * the scrunched samples of oracle_scrunch: the paper applies the tree to
 * scrunched data for the larger DMs in the same way). */
int oracle_tree_imposed_values(const uint32_t* x, int64_t nsamps, int nchans, int k, int slope,
                               uint32_t* out, const int32_t* mask)
{
    return tree_steps(NULL, x, nsamps, nchans, 0, k, slope, out, mask);
}

/* Stage 2 of the piecewise linear tree (Section 3, eq. combining_subbands):
 * with sub-bands of nsub = 2^k channels (sub-band n starting at channel
 * v_n = n*nsub; v_{nsb} = nchans is the channel just past the band),
 *   d'_n(d)  = round(DM(d) [DeltaT(v_{n+1}) - DeltaT(v_n)])
 *   dt''_n(d) = round(DM(d) * sum over m < n of [DeltaT(v_{m+1}) - DeltaT(v_m)])
 * (the sum runs over the sub-bands before n, so each sub-band's series, which
 * the tree aligns on its first channel, is placed at the delay of that
 * channel), both evaluated in binary64 in this order, and
 *   D[d][t] = sum over n of S[n*nsub + d'_n(d)][t + dt''_n(d)]
 * for t < len1 - (largest dt''), S being the k-step tree output of length
 * len1 (oracle_tree_combine).  This function returns the tables dprime and
 * dpp [ndm][nsb]; d'_n(d) may reach nsub and beyond (DMs past the piecewise
 * diagonal, which oracle_tree_combine_passes serves). */
int oracle_tree_dm_tables(int nchans, double dt, double f_top, double df, int nsub,
                          const double* dms, int ndm, int32_t* dprime, int32_t* dpp)
{
    if (!dms || !dprime || !dpp || nsub <= 0 || nchans % nsub) return ORACLE_BAD_ARG;
    if (oracle_check_params(nchans, dt, f_top, df, 8) != ORACLE_OK) return ORACLE_BAD_ARG;
    if (!(f_top + (double)nchans * df > 0.0)) return ORACLE_BAD_ARG;
    const int nsb = nchans / nsub;
    const double inv_top2 = 1.0 / (f_top * f_top);
    const double scale = ORACLE_K_DM / dt;
    for (int d = 0; d < ndm; ++d) {
        double acc = 0.0;
        for (int n = 0; n < nsb; ++n) {
            const double fa = f_top + (double)(n * nsub) * df;
            const double fb = f_top + (double)((n + 1) * nsub) * df;
            const double step = scale * (1.0 / (fb * fb) - inv_top2) - scale * (1.0 / (fa * fa) - inv_top2);
            const double dp = round(dms[d] * step);
            const double dd = round(dms[d] * acc);
            if (!(dp >= 0.0) || dp > 2.0e9 || !(dd >= 0.0) || dd > 2.0e9) return ORACLE_BAD_ARG;
            dprime[(size_t)d * nsb + n] = (int32_t)dp;
            dpp[(size_t)d * nsb + n] = (int32_t)dd;
            acc += step;
        }
    }
    return ORACLE_OK;
}

/* The same tables for DMs up to the piecewise diagonal: every d'_n(d) must be
 * below nsub. */
int oracle_tree_combine_tables(int nchans, double dt, double f_top, double df, int nsub,
                               const double* dms, int ndm, int32_t* dprime, int32_t* dpp)
{
    const int rc = oracle_tree_dm_tables(nchans, dt, f_top, df, nsub, dms, ndm, dprime, dpp);
    if (rc != ORACLE_OK) return rc;
    for (size_t i = 0; i < (size_t)ndm * (size_t)(nchans / nsub); ++i)
        if (dprime[i] >= nsub) return ORACLE_BAD_ARG;
    return ORACLE_OK;
}

int oracle_tree_combine(const uint32_t* S, int nchans, int64_t len1, int nsub,
                        const int32_t* dprime, const int32_t* dpp, int ndm, int64_t nout,
                        uint32_t* out)
{
    if (!S || !dprime || !dpp || !out || nsub <= 0 || nchans % nsub || nout <= 0) return ORACLE_BAD_ARG;
    const int nsb = nchans / nsub;
    for (int d = 0; d < ndm; ++d)
        for (int n = 0; n < nsb; ++n)
            if (nout + dpp[(size_t)d * nsb + n] > len1 || dprime[(size_t)d * nsb + n] >= nsub)
                return ORACLE_BAD_ARG;
#pragma omp parallel for schedule(dynamic, 1)
    for (int d = 0; d < ndm; ++d) {
        uint32_t* row = out + (size_t)d * (size_t)nout;
        for (int64_t t = 0; t < nout; ++t) {
            uint32_t sum = 0;
            for (int n = 0; n < nsb; ++n) {
                const int32_t dp = dprime[(size_t)d * nsb + n];
                sum += S[((size_t)n * nsub + dp) * (size_t)len1 + (size_t)(t + dpp[(size_t)d * nsb + n])];
            }
            row[t] = sum;
        }
    }
    return ORACLE_OK;
}

/* Stage 2 over several passes (Section 3, computing larger DMs): S holds
 * npass stage-1 outputs [npass][nchans][len1], pass p taken with an imposed
 * slope of p samples per channel (oracle_tree_imposed, truncated to len1).
 * Sub-band n of trial d reads pass p = d'_n(d) / nsub at row
 * n*nsub + d'_n(d) mod nsub, placed at dt''_n(d) as before:
 *   D[d][t] = sum over n of S[p][n*nsub + d'_n(d) - p*nsub][t + dt''_n(d)]. */
int oracle_tree_combine_passes(const uint32_t* S, int npass, int nchans, int64_t len1, int nsub,
                               const int32_t* dprime, const int32_t* dpp, int ndm, int64_t nout,
                               uint32_t* out)
{
    if (!S || !dprime || !dpp || !out || npass <= 0 || nsub <= 0 || nchans % nsub || nout <= 0)
        return ORACLE_BAD_ARG;
    const int nsb = nchans / nsub;
    for (int d = 0; d < ndm; ++d)
        for (int n = 0; n < nsb; ++n)
            if (nout + dpp[(size_t)d * nsb + n] > len1 || dprime[(size_t)d * nsb + n] / nsub >= npass)
                return ORACLE_BAD_ARG;
#pragma omp parallel for schedule(dynamic, 1)
    for (int d = 0; d < ndm; ++d) {
        uint32_t* row = out + (size_t)d * (size_t)nout;
        for (int64_t t = 0; t < nout; ++t) {
            uint32_t sum = 0;
            for (int n = 0; n < nsb; ++n) {
                const int32_t dp = dprime[(size_t)d * nsb + n];
                const int p = dp / nsub;
                const size_t r = (size_t)p * nchans + (size_t)n * nsub + (size_t)(dp % nsub);
                sum += S[r * (size_t)len1 + (size_t)(t + dpp[(size_t)d * nsb + n])];
            }
            row[t] = sum;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Output bit depth (Section 4: the final output is written with a chosen
 * number of bits per sample).  The paper does not say how a sum is brought
 * to 8 or 16 bits; the reading fixed here is a right shift by `shift` bits
 * followed by saturation at the largest value of the width:
 *   out = min(sum >> shift, 2^nbits - 1),
 * so an output is exact whenever the shifted sum fits.
 * ------------------------------------------------------------------------ */
int oracle_reduce_output(const uint32_t* sums, int64_t n, int nbits, int shift, void* out)
{
    if (!sums || !out || n < 0 || shift < 0 || shift > 31) return ORACLE_BAD_ARG;
    if (nbits != 8 && nbits != 16 && nbits != 32) return ORACLE_BAD_ARG;
    const uint64_t top = nbits == 32 ? 0xFFFFFFFFull : ((1ull << nbits) - 1ull);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t v = (uint64_t)(sums[i] >> shift);
        if (v > top) v = top;
        if (nbits == 8) ((uint8_t*)out)[i] = (uint8_t)v;
        else if (nbits == 16) ((uint16_t*)out)[i] = (uint16_t)v;
        else ((uint32_t*)out)[i] = (uint32_t)v;
    }
    return ORACLE_OK;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
