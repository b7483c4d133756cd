/*
 * snn_oracle.c -- plain FP64 CPU reference of the minibatched clock-driven
 * spiking network (Saunders et al., "Minibatch Processing in Spiking Neural
 * Networks", AAAI-20).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * What it computes (all floating point in double precision):
 *   - per-sample state (voltages, refractory counters, traces, previous
 *     spikes) duplicated B times; weights and adaptive thresholds held once
 *     and updated with a batch reduction (Implementation section);
 *   - Poisson input spikes, rate = pixel / 255 * max_rate (Unsupervised
 *     Learning section), drawn as one Bernoulli trial per (sample, input,
 *     step) from Philox4x64-10 keyed by (seed, sample id, local step);
 *   - LIF layers (Scaling section) and the adaptive-threshold excitatory layer
 *     with one-to-one exc->inh and all-but-self inh->exc inhibition
 *     (Unsupervised Learning section);
 *   - online STDP from nearest-spike traces, reduced over the batch by sum,
 *     mean or per-synapse maximum (Reduction methods section; Fig. 3 text),
 *     by the signed maximum of the per-sample changes (a variant), or by the
 *     soft maximum tau log((1/B) sum_b exp(z_b / tau)) (a user-chosen
 *     reduction, which the section allows, between the mean and the max),
 *     clamp to [w_min, w_max] and per-column normalisation to a fixed sum
 *     (Unsupervised Learning section).
 * Readings of points the paper leaves open are listed in the design notes:
 * exact exponential decay, current-based synapses, input discarded while
 * refractory, >= threshold test, one-step delay on recurrent connections,
 * traces updated before the weight change, update -> clamp -> normalise every
 * learning step, theta decays and grows only while learning.
 *
 * Loops are written in the order the definition reads.  The feed-forward sum
 * skips inputs that did not spike (adding an exact zero changes nothing); the
 * batch reductions visit every sample.  OpenMP splits only independent output
 * elements, so every sum keeps one fixed order.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies on a
 * 4-word counter, the 2-word key bumped by two Weyl constants between rounds. */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2E7470EE14C6C93ULL
#define ORC_PHILOX_M1 0xCA5A826395121157ULL
#define ORC_PHILOX_W0 0x9E3779B97F4A7C15ULL
#define ORC_PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)ORC_PHILOX_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)ORC_PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The 32-bit uniform that decides input i of sample `id` at local step t:
 * counter (i / 8, t, id, 0), key (seed, 0); the four 64-bit outputs are read
 * as eight 32-bit words, low half first. */
/* Host threads the parallel loops use (timing only; results do not depend
 * on it: every parallel loop writes disjoint outputs). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_threads(void) { return omp_get_max_threads(); }

uint32_t orc_uniform32(uint64_t seed, uint64_t id, uint64_t t, uint64_t i)
{
    uint64_t ctr[4] = {i / 8, t, id, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t w = out[(i % 8) / 2];
    return (i % 2 == 0) ? (uint32_t)(w & 0xffffffffULL) : (uint32_t)(w >> 32);
}

/* ------------------------------------------------------------------------ */
/* configuration                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    double v_rest, v_reset, v_thresh, tau_ms;
    int32_t refrac_steps, adaptive;
    double theta_plus, tau_theta_ms;
} orc_lif;

typedef struct {
    int32_t n_in, n_exc, n_inh;      /* n_inh = 0: no inhibitory layer      */
    int32_t uniform_rate, learn;     /* uniform_rate: every input max_rate  */
    int32_t trace_additive, reduce;  /* reduce: 0 sum, 1 mean, 2 max, 3 signed max, 4 soft max */
    int32_t precision;               /* operand rounding, see orc_quantize  */
    double dt_ms, max_rate_hz;
    orc_lif exc, inh;
    double w_ei, w_ie;
    double nu_pre, nu_post, tau_pre_ms, tau_post_ms, w_min, w_max, norm;
    uint64_t seed;
    int32_t norm_per_run;            /* 1: normalise after a run's last step only */
    double reduce_tau;               /* temperature of the soft maximum (reduce 4) */
} orc_config;

/* ------------------------------------------------------------------------ */
/* Operand precision of the two contractions.  The synaptic contraction and  */
/* the STDP products multiply exact 0/1 spikes by a weight or a trace; in    */
/* the reduced-precision forms that weight or trace enters rounded to        */
/* bfloat16 or to OCP FP8 E4M3, while sums stay wide and the master weights  */
/* stay full precision.  The rounding starts from the value's single-        */
/* precision form (the precision the kernels hold it in), so both sides take */
/* the same rounding decision.                                                */
/*   0  none (FP64 here)                                                      */
/*   1  bfloat16: 8 significant bits, FP32 exponent range                     */
/*   2  E4M3 (OCP FP8): 4 significant bits, exponent bias 7, smallest normal  */
/*      2^-6, subnormal spacing 2^-9, largest finite 448 (saturating here)    */
/* Both round to nearest, ties to even.                                       */
/* ------------------------------------------------------------------------ */
static double round_to_grid(double x, int mant_bits, int min_exp)
{
    /* nearest multiple of 2^(e - mant_bits + 1), e = max(floor(log2|x|), min_exp) */
    double a = fabs(x);
    if (a == 0.0 || !isfinite(a)) return x;
    int e;
    frexp(a, &e);        /* a = m 2^e, m in [0.5, 1): floor(log2 a) = e - 1 */
    e -= 1;
    if (e < min_exp) e = min_exp;
    double ulp = ldexp(1.0, e - mant_bits + 1);
    double q = nearbyint(a / ulp) * ulp; /* default rounding: nearest, ties to even */
    return x < 0 ? -q : q;
}

double orc_quantize(double x, int precision)
{
    if (precision == 0) return x;
    double f = (double)(float)x;
    if (precision == 1) return round_to_grid(f, 8, -126);
    double q = round_to_grid(f, 4, -6);
    if (q > 448.0) q = 448.0;
    if (q < -448.0) q = -448.0;
    return q;
}

/* Spike probability per step as a 32-bit threshold: a spike happens when the
 * uniform word is below thr.  Rate for pixel p is p/255 * max_rate (Hz), so
 * the per-step probability is rate * dt.  thr = floor(prob * 2^32). */
uint32_t orc_threshold(const orc_config *c, int pixel)
{
    double prob = c->uniform_rate ? c->max_rate_hz * c->dt_ms / 1000.0
                                  : (double)pixel * c->max_rate_hz * c->dt_ms / (255.0 * 1000.0);
    double thr = floor(prob * 4294967296.0);
    if (thr < 0.0) thr = 0.0;
    if (thr > 4294967295.0) thr = 4294967295.0;
    return (uint32_t)thr;
}

/* The batch reduction of one synapse's (or neuron's) B contributions:
 * sum, mean, maximum, or (mode 4) the soft maximum with temperature tau,
 * tau log((1/B) sum_b exp(terms[b] / tau)) (the log-mean-exp). */
static double reduce_terms(const double *terms, int B, int mode, double tau)
{
    if (mode == 4) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += exp(terms[b] / tau);
        return tau * log(s / (double)B);
    }
    if (mode == 2) {
        double m = terms[0];
        for (int b = 1; b < B; ++b)
            if (terms[b] > m) m = terms[b];
        return m;
    }
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += terms[b];
    return mode == 1 ? s / (double)B : s;
}

/* One LIF population update for one sample.  Returns spikes in s_out. */
static void lif_step(const orc_lif *p, int n, double alpha, double *v, int32_t *r,
                     const double *I, const double *theta, uint8_t *s_out)
{
    for (int j = 0; j < n; ++j) {
        /* exact exponential relaxation towards rest over one step */
        v[j] = p->v_rest + (v[j] - p->v_rest) * alpha;
        if (r[j] > 0) {
            /* refractory: input discarded, counter runs down */
            r[j] -= 1;
            s_out[j] = 0;
            continue;
        }
        v[j] += I[j];
        double th = p->v_thresh + (theta ? theta[j] : 0.0);
        if (v[j] >= th) {
            s_out[j] = 1;
            v[j] = p->v_reset;
            r[j] = p->refrac_steps;
        } else {
            s_out[j] = 0;
        }
    }
}

/*
 * Run T steps of a batch of B samples, starting from the state passed in
 * (episodic reset is the caller's job: fill v with v_rest and the rest with
 * zeros).  Sample b's local step numbers are t_start[b] .. t_start[b]+T-1
 * (all equal unless the batch was re-formed without a reset).
 *
 * Inputs:   images  B x n_in uint8 (ignored when uniform_rate or forced_in)
 *           ids     B sample ids
 *           forced_in  optional B x T x n_in 0/1 input raster used instead of
 *                      the Poisson encoder
 * In/out:   W (n_in x n_exc, row-major), theta (n_exc), state arrays
 * Records (each optional, NULL to skip):
 *           rec_in  B x T x n_in, rec_exc B x T x n_exc, rec_inh B x T x n_inh,
 *           rec_v_exc B x T x n_exc, rec_v_inh B x T x n_inh,
 *           counts  B x n_exc (accumulated),
 *           rec_theta T x n_exc (theta after each step)
 * Returns 0, or -1 on an invalid configuration, -2 on allocation failure.
 */
int orc_run(const orc_config *c, int B, int T, const int64_t *t_start,
            const uint8_t *images, const uint64_t *ids, const uint8_t *forced_in,
            double *W, double *theta,
            double *v_exc, double *v_inh, int32_t *r_exc, int32_t *r_inh,
            double *x_pre, double *x_post, uint8_t *s_exc_prev, uint8_t *s_inh_prev,
            uint8_t *rec_in, uint8_t *rec_exc, uint8_t *rec_inh,
            double *rec_v_exc, double *rec_v_inh, uint32_t *counts, double *rec_theta)
{
    const int n_in = c->n_in, n_exc = c->n_exc, n_inh = c->n_inh;
    if (B <= 0 || T < 0 || n_in <= 0 || n_exc <= 0 || n_inh < 0) return -1;
    if (n_inh > 0 && n_inh != n_exc) return -1; /* one-to-one exc->inh */

    const double alpha_exc = exp(-c->dt_ms / c->exc.tau_ms);
    const double alpha_inh = exp(-c->dt_ms / c->inh.tau_ms);
    const double beta = exp(-c->dt_ms / c->exc.tau_theta_ms);
    const double lam_pre = exp(-c->dt_ms / c->tau_pre_ms);
    const double lam_post = exp(-c->dt_ms / c->tau_post_ms);
    const int adaptive = c->exc.adaptive != 0;
    const int prec = c->precision;
    if (prec < 0 || prec > 2) return -1;

    uint32_t thr_lut[256];
    for (int p = 0; p < 256; ++p) thr_lut[p] = orc_threshold(c, p);

    uint8_t *s_in = calloc((size_t)B * n_in, 1);
    uint8_t *s_exc = calloc((size_t)B * n_exc, 1);
    uint8_t *s_inh = calloc((size_t)B * (n_inh > 0 ? n_inh : 1), 1);
    double *I_exc = calloc((size_t)B * n_exc, sizeof(double));
    double *I_inh = calloc((size_t)B * (n_inh > 0 ? n_inh : 1), sizeof(double));
    if (!s_in || !s_exc || !s_inh || !I_exc || !I_inh) {
        free(s_in); free(s_exc); free(s_inh); free(I_exc); free(I_inh);
        return -2;
    }

    for (int k = 0; k < T; ++k) {
        /* 1. input spikes (sample b at its own local step t_start[b] + k) */
#pragma omp parallel for schedule(static)
        for (int b = 0; b < B; ++b) {
            const uint64_t t = (uint64_t)(t_start[b] + k);
            for (int i = 0; i < n_in; ++i) {
                uint8_t s;
                if (forced_in) {
                    s = forced_in[((size_t)b * T + k) * n_in + i] ? 1 : 0;
                } else {
                    uint32_t thr = c->uniform_rate ? thr_lut[0] : thr_lut[images[(size_t)b * n_in + i]];
                    s = orc_uniform32(c->seed, ids[b], t, (uint64_t)i) < thr;
                }
                s_in[(size_t)b * n_in + i] = s;
            }
        }

        /* 2. currents: feed-forward (same step) and recurrent (previous step) */
#pragma omp parallel for schedule(static)
        for (int b = 0; b < B; ++b) {
            double *Ie = I_exc + (size_t)b * n_exc;
            for (int j = 0; j < n_exc; ++j) Ie[j] = 0.0;
            for (int i = 0; i < n_in; ++i) {
                if (!s_in[(size_t)b * n_in + i]) continue;
                const double *row = W + (size_t)i * n_exc;
                for (int j = 0; j < n_exc; ++j) Ie[j] += orc_quantize(row[j], prec);
            }
            if (n_inh > 0) {
                const uint8_t *si = s_inh_prev + (size_t)b * n_inh;
                const uint8_t *se = s_exc_prev + (size_t)b * n_exc;
                long count = 0;
                for (int q = 0; q < n_inh; ++q) count += si[q];
                for (int j = 0; j < n_exc; ++j)
                    Ie[j] += c->w_ie * (double)(count - si[j]);
                double *Ii = I_inh + (size_t)b * n_inh;
                for (int j = 0; j < n_inh; ++j) Ii[j] = c->w_ei * (double)se[j];
            }
        }

        /* 3. adaptive threshold decay (only while learning) */
        if (c->learn && adaptive)
            for (int j = 0; j < n_exc; ++j) theta[j] *= beta;

        /* 4. neuron updates */
#pragma omp parallel for schedule(static)
        for (int b = 0; b < B; ++b) {
            lif_step(&c->exc, n_exc, alpha_exc, v_exc + (size_t)b * n_exc, r_exc + (size_t)b * n_exc,
                     I_exc + (size_t)b * n_exc, adaptive ? theta : NULL, s_exc + (size_t)b * n_exc);
            if (n_inh > 0)
                lif_step(&c->inh, n_inh, alpha_inh, v_inh + (size_t)b * n_inh, r_inh + (size_t)b * n_inh,
                         I_inh + (size_t)b * n_inh, NULL, s_inh + (size_t)b * n_inh);
        }

        if (c->learn) {
            /* 5. traces: decay, then set (or add) on a spike */
#pragma omp parallel for schedule(static)
            for (int b = 0; b < B; ++b) {
                for (int i = 0; i < n_in; ++i) {
                    double *x = x_pre + (size_t)b * n_in + i;
                    *x *= lam_pre;
                    if (s_in[(size_t)b * n_in + i]) *x = c->trace_additive ? *x + 1.0 : 1.0;
                }
                for (int j = 0; j < n_exc; ++j) {
                    double *x = x_post + (size_t)b * n_exc + j;
                    *x *= lam_post;
                    if (s_exc[(size_t)b * n_exc + j]) *x = c->trace_additive ? *x + 1.0 : 1.0;
                }
            }

            /* 6-7. batch-reduced weight change, clamp.  P: potentiation on a
             * post spike from the pre trace; D: depression on a pre spike from
             * the post trace; each reduced over the batch on its own, visiting
             * the samples in order b = 0 .. B-1.  Signed max (mode 3) instead
             * takes, per synapse, the largest of the B per-sample changes
             * nu_post tp - nu_pre td (0 for a sample with neither spike).  The
             * soft maximum (mode 4) sums exp(term / tau) over all B terms,
             * zeros included, and takes tau log(sum / B). */
#pragma omp parallel
            {
                double *P = malloc(sizeof(double) * (size_t)n_exc);
                double *D = malloc(sizeof(double) * (size_t)n_exc);
                double *M = malloc(sizeof(double) * (size_t)n_exc);
#pragma omp for schedule(static)
                for (int i = 0; i < n_in; ++i) {
                    for (int b = 0; b < B; ++b) {
                        const double xp = x_pre[(size_t)b * n_in + i];
                        const int sp = s_in[(size_t)b * n_in + i];
                        const uint8_t *se = s_exc + (size_t)b * n_exc;
                        const double *xq = x_post + (size_t)b * n_exc;
                        for (int j = 0; j < n_exc; ++j) {
                            double tp = se[j] ? orc_quantize(xp, prec) : 0.0;
                            double td = sp ? orc_quantize(xq[j], prec) : 0.0;
                            if (c->reduce == 3) {
                                double dw = c->nu_post * tp - c->nu_pre * td;
                                if (b == 0 || dw > M[j]) M[j] = dw;
                            }
                            if (c->reduce == 4) {
                                tp = exp(tp / c->reduce_tau);
                                td = exp(td / c->reduce_tau);
                            }
                            if (b == 0) {
                                P[j] = tp;
                                D[j] = td;
                            } else if (c->reduce == 2) {
                                P[j] = tp > P[j] ? tp : P[j];
                                D[j] = td > D[j] ? td : D[j];
                            } else {
                                P[j] += tp;
                                D[j] += td;
                            }
                        }
                    }
                    for (int j = 0; j < n_exc; ++j) {
                        double Pj = c->reduce == 1 ? P[j] / (double)B : P[j];
                        double Dj = c->reduce == 1 ? D[j] / (double)B : D[j];
                        if (c->reduce == 4) {
                            Pj = c->reduce_tau * log(P[j] / (double)B);
                            Dj = c->reduce_tau * log(D[j] / (double)B);
                        }
                        double w = c->reduce == 3 ? W[(size_t)i * n_exc + j] + M[j]
                                                  : W[(size_t)i * n_exc + j] + c->nu_post * Pj - c->nu_pre * Dj;
                        if (w < c->w_min) w = c->w_min;
                        if (w > c->w_max) w = c->w_max;
                        W[(size_t)i * n_exc + j] = w;
                    }
                }
                free(P);
                free(D);
                free(M);
            }

            /* 7b. column normalisation: the weights into each post neuron
             * sum to `norm` (skipped for an all-zero column); every learning
             * step, or (the cheaper variant) after the run's last step only */
            if (c->norm > 0.0 && (!c->norm_per_run || k == T - 1)) {
#pragma omp parallel for schedule(static)
                for (int j = 0; j < n_exc; ++j) {
                    double cs = 0.0;
                    for (int i = 0; i < n_in; ++i) cs += W[(size_t)i * n_exc + j];
                    if (cs > 0.0) {
                        double scale = c->norm / cs;
                        for (int i = 0; i < n_in; ++i) W[(size_t)i * n_exc + j] *= scale;
                    }
                }
            }

            /* 8. adaptive threshold increment, batch-reduced like the weights */
            if (adaptive) {
                double *terms = malloc(sizeof(double) * (size_t)B);
                for (int j = 0; j < n_exc; ++j) {
                    for (int b = 0; b < B; ++b) terms[b] = (double)s_exc[(size_t)b * n_exc + j];
                    theta[j] += c->exc.theta_plus * reduce_terms(terms, B, c->reduce == 3 ? 2 : c->reduce,
                                                                 c->reduce_tau);
                }
                free(terms);
            }
        }

        /* 9. record, then the current spikes become the previous spikes */
        for (int b = 0; b < B; ++b) {
            size_t row = (size_t)b * T + k;
            if (rec_in) memcpy(rec_in + row * n_in, s_in + (size_t)b * n_in, (size_t)n_in);
            if (rec_exc) memcpy(rec_exc + row * n_exc, s_exc + (size_t)b * n_exc, (size_t)n_exc);
            if (rec_inh && n_inh > 0) memcpy(rec_inh + row * n_inh, s_inh + (size_t)b * n_inh, (size_t)n_inh);
            if (rec_v_exc) memcpy(rec_v_exc + row * n_exc, v_exc + (size_t)b * n_exc, sizeof(double) * n_exc);
            if (rec_v_inh && n_inh > 0) memcpy(rec_v_inh + row * n_inh, v_inh + (size_t)b * n_inh, sizeof(double) * n_inh);
            if (counts)
                for (int j = 0; j < n_exc; ++j) counts[(size_t)b * n_exc + j] += s_exc[(size_t)b * n_exc + j];
        }
        if (rec_theta) memcpy(rec_theta + (size_t)k * n_exc, theta, sizeof(double) * n_exc);
        memcpy(s_exc_prev, s_exc, (size_t)B * n_exc);
        if (n_inh > 0) memcpy(s_inh_prev, s_inh, (size_t)B * n_inh);
    }

    free(s_in); free(s_exc); free(s_inh); free(I_exc); free(I_inh);
    return 0;
}
