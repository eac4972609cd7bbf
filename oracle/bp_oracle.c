/*
 * TEST INFRASTRUCTURE -- the fp64 CPU oracle for the LDPC part of the
 * slice-reconciliation hot path.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product path
 * never does.  It shares no code, header or table with the HIP library.
 *
 * Conventions (the paper names the belief-propagation decoder but fixes no
 * variant; these are the readings taken here):
 *   - an LLR is ln P(bit = 0) / P(bit = 1); hard decision b = 1 iff L < 0;
 *   - sign(x) = -1 iff x < 0 (so -0.0 counts as +);
 *   - syndrome decoding: every check-to-variable message of check c is
 *     multiplied by (1 - 2 s_c), s_c being the syndrome bit Bob sends
 *     (Sec. II Step 5, Sec. III-B steps 2-4);
 *   - flooding schedule (orc_decode): all checks, then all variables, per
 *     iteration; the layered schedule (orc_decode_layered) updates groups of
 *     rows one after another within an iteration;
 *   - the syndrome of the hard decisions is tested before the first
 *     iteration and after every iteration (failure detection, Sec. II Step 5).
 *
 * orc_flood_step and orc_layered_step run a single iteration from a given
 * state, so that the fp64 definitions and the binary32 forms can be compared
 * one step at a time.
 *
 * Every function below is plain loops in double precision, written to be
 * read against its definition rather than to be fast.  OpenMP splits the
 * independent frames (sub-blocks, Sec. III-A) across host threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SP 0
#define ORC_NMS 1

/* ------------------------------------------------------------------------ */
/* syndrome s_c = XOR_{v in N(c)} b_v   (Sec. II Step 5; Sec. III-B step 2)  */
/* ------------------------------------------------------------------------ */
int orc_syndrome(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                 int32_t F, const uint8_t* bits, const uint8_t* s_ref,
                 uint8_t* s_out, int32_t* n_unsat)
{
    for (int32_t f = 0; f < F; ++f) {
        const uint8_t* b = bits + (int64_t)f * n;
        int32_t u = 0;
        for (int32_t c = 0; c < m; ++c) {
            int s = 0;
            for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) s ^= (b[col_idx[e]] & 1);
            if (s_out) s_out[(int64_t)f * m + c] = (uint8_t)s;
            int ref = s_ref ? (s_ref[(int64_t)f * m + c] & 1) : 0;
            u += (s != ref);
        }
        if (n_unsat) n_unsat[f] = u;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* binary16 storage emulation: round-to-nearest-even to the IEEE half grid,   */
/* saturating at +-65504 (largest finite half).                               */
/* ------------------------------------------------------------------------ */
double orc_round_half(double x)
{
    if (isnan(x)) return x;
    double a = fabs(x);
    if (a >= 65504.0) return copysign(65504.0, x);
    if (a == 0.0) return x;
    int e;
    frexp(a, &e);                 /* a = f * 2^e, f in [0.5, 1) -> exponent of a is e-1 */
    int ex = e - 1;
    if (ex < -14) ex = -14;       /* subnormal halves share the 2^-24 spacing */
    double ulp = ldexp(1.0, ex - 10);
    double r = nearbyint(a / ulp) * ulp;   /* default rounding mode: nearest-even */
    if (r > 65504.0) r = 65504.0;
    return copysign(r, x);
}

/* phi(x) = -ln tanh(x/2) = ln(1 + 2/(e^x - 1)), phi(0) = +inf, phi(+inf) = 0. */
static double phi(double x)
{
    if (x == 0.0) return INFINITY;
    if (isinf(x)) return 0.0;
    return log1p(2.0 / expm1(x));
}

static inline int neg(double x) { return x < 0.0; }

/* Column view of a CSR matrix: for variable v, the CSR edge ids of its checks
 * in ascending check order. */
typedef struct { int32_t* ptr; int32_t* edge; } colview;

static colview make_colview(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx)
{
    colview cv;
    int64_t E = row_ptr[m];
    cv.ptr = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    cv.edge = (int32_t*)malloc((size_t)(E > 0 ? E : 1) * sizeof(int32_t));
    for (int64_t e = 0; e < E; ++e) cv.ptr[col_idx[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) cv.ptr[v + 1] += cv.ptr[v];
    int32_t* fill = (int32_t*)malloc((size_t)n * sizeof(int32_t) + 1);
    for (int32_t v = 0; v < n; ++v) fill[v] = cv.ptr[v];
    for (int32_t c = 0; c < m; ++c)                      /* rows ascending -> checks ascending */
        for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) cv.edge[fill[col_idx[e]]++] = e;
    free(fill);
    return cv;
}

static void free_colview(colview* cv) { free(cv->ptr); free(cv->edge); }

/* Number of checks whose parity over the hard decisions differs from s.  A
 * check touching a NaN posterior counts as unsatisfied, so that a frame fed a
 * NaN LLR can never be reported as decoded. */
static int32_t count_unsat(int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                           const double* L, const uint8_t* s)
{
    int32_t u = 0;
    for (int32_t c = 0; c < m; ++c) {
        int p = s ? (s[c] & 1) : 0;
        int nan = 0;
        for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
            p ^= neg(L[col_idx[e]]);
            nan |= isnan(L[col_idx[e]]) ? 1 : 0;
        }
        u += p | nan;
    }
    return u;
}

/*
 * Flooding belief propagation on F frames that share one parity-check matrix.
 *
 * algo = ORC_SP (sum-product):
 *   c2v_e = (1 - 2 s_c) * prod_{k != e} sign(v2c_k) * phi( sum_{k != e} phi(|v2c_k|) )
 *   with every v2c first clamped to [-clamp, clamp].
 * algo = ORC_NMS (normalized min-sum):
 *   c2v_e = w * (1 - 2 s_c) * prod_{k != e} sign(v2c_k) * min_{k != e} |v2c_k|,
 *   w = weights[t * n_types + type_e] when weights != NULL, else alpha.
 * Both:  v2c_e = L_ch[v] + sum_{c' in N(v), c' != c} c2v_{c'}  (extrinsic);
 *        L_post[v] = L_ch[v] + sum_{c in N(v)} c2v_c.
 * store_half != 0 rounds every stored c2v to binary16 (nearest-even, saturating).
 *
 * Iteration t = 0..T: the hard decisions of L_post(t) are tested against the
 * syndrome (L_post(0) = L_ch); with early_stop the frame ends at the first t
 * with no unsatisfied check; otherwise (or if never satisfied) it ends at T.
 * Outputs: bits, L_post, iters = that t, ok = [no unsatisfied check at t].
 * Optional traces ([F][T+1][n] / [F][T+1]): L_post(t), the scale
 * |L_ch| + sum |c2v| of each posterior sum, and the unsatisfied-check count;
 * entries after a frame's stop are left untouched.
 *
 * prec32 != 0 takes every step in binary32 instead: each result of an add,
 * subtract, multiply or phi is rounded to the nearest float (computing in
 * double and rounding once is exact for these operations since 53 >= 2*24+2),
 * the posterior is accumulated from L_ch in ascending check order, and the
 * extrinsic message is formed as L_post - c2v, which equals the sum above in
 * exact arithmetic.  This is the precision in which a binary32 decoder takes
 * its rounding-to-binary16 and minimum-selection decisions.
 */
static inline double rnd(int prec32, double x) { return prec32 ? (double)(float)x : x; }

int orc_decode(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
               const uint8_t* edge_type, int32_t n_types,
               int32_t F, const double* llr, const uint8_t* syn,
               int32_t algo, int32_t T, int32_t early_stop, int32_t store_half, int32_t prec32,
               double alpha, const double* weights, double clamp,
               uint8_t* bits, double* post, int32_t* iters, uint8_t* ok,
               double* trace, double* trace_scale, int32_t* trace_unsat)
{
    if (n <= 0 || m < 0 || F < 0 || T < 0) return -1;
    const int64_t E = row_ptr[m];
    colview cv = make_colview(n, m, row_ptr, col_idx);
    int32_t maxdeg = 0;
    for (int32_t c = 0; c < m; ++c)
        if (row_ptr[c + 1] - row_ptr[c] > maxdeg) maxdeg = row_ptr[c + 1] - row_ptr[c];

#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
        const double* Lch = llr + (int64_t)f * n;
        const uint8_t* s = syn ? syn + (int64_t)f * m : NULL;
        double* c2v = (double*)calloc((size_t)(E > 0 ? E : 1), sizeof(double));
        double* v2c = (double*)malloc((size_t)(E > 0 ? E : 1) * sizeof(double));
        double* Lp = (double*)malloc((size_t)n * sizeof(double));
        double* mag = (double*)malloc((size_t)(maxdeg > 0 ? maxdeg : 1) * sizeof(double));
        for (int32_t v = 0; v < n; ++v) Lp[v] = rnd(prec32, Lch[v]);

        int32_t t = 0;
        for (;;) {
            int32_t u = count_unsat(m, row_ptr, col_idx, Lp, s);
            if (trace) memcpy(trace + ((int64_t)f * (T + 1) + t) * n, Lp, (size_t)n * sizeof(double));
            if (trace_scale) {
                double* sc = trace_scale + ((int64_t)f * (T + 1) + t) * n;
                for (int32_t v = 0; v < n; ++v) {
                    double a = fabs(Lch[v]);
                    if (t > 0)
                        for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) a += fabs(c2v[cv.edge[k]]);
                    sc[v] = a;
                }
            }
            if (trace_unsat) trace_unsat[(int64_t)f * (T + 1) + t] = u;
            if ((early_stop && u == 0) || t == T) {
                iters[f] = t;
                ok[f] = (uint8_t)(u == 0);
                break;
            }

            /* variable-to-check: extrinsic sums */
            for (int32_t v = 0; v < n; ++v) {
                for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) {
                    double a;
                    if (prec32) {
                        a = rnd(1, Lp[v] - c2v[cv.edge[k]]);
                    } else {
                        a = Lch[v];
                        for (int32_t k2 = cv.ptr[v]; k2 < cv.ptr[v + 1]; ++k2)
                            if (k2 != k) a += c2v[cv.edge[k2]];
                    }
                    v2c[cv.edge[k]] = a;
                }
            }

            /* check-to-variable */
            for (int32_t c = 0; c < m; ++c) {
                const int32_t e0 = row_ptr[c], e1 = row_ptr[c + 1];
                const double ssign = (s && (s[c] & 1)) ? -1.0 : 1.0;
                for (int32_t e = e0; e < e1; ++e) {
                    double x = v2c[e];
                    if (algo == ORC_SP) {
                        if (x > clamp) x = clamp;
                        if (x < -clamp) x = -clamp;
                    }
                    mag[e - e0] = x;
                }
                for (int32_t e = e0; e < e1; ++e) {
                    double sg = ssign;
                    for (int32_t k = e0; k < e1; ++k)
                        if (k != e && neg(mag[k - e0])) sg = -sg;
                    double out;
                    if (algo == ORC_SP) {
                        double acc = 0.0;
                        for (int32_t k = e0; k < e1; ++k)
                            if (k != e) acc = rnd(prec32, acc + rnd(prec32, phi(fabs(mag[k - e0]))));
                        out = sg * rnd(prec32, phi(acc));
                    } else {
                        double mn = INFINITY;
                        for (int32_t k = e0; k < e1; ++k)
                            if (k != e && fabs(mag[k - e0]) < mn) mn = fabs(mag[k - e0]);
                        double w = weights ? weights[(int64_t)t * n_types + (edge_type ? edge_type[e] : 0)] : alpha;
                        out = rnd(prec32, rnd(prec32, w) * (sg * mn));
                    }
                    c2v[e] = store_half ? orc_round_half(out) : out;
                }
            }

            /* posteriors */
            for (int32_t v = 0; v < n; ++v) {
                double a = rnd(prec32, Lch[v]);
                for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) a = rnd(prec32, a + c2v[cv.edge[k]]);
                Lp[v] = a;
            }
            ++t;
        }
        for (int32_t v = 0; v < n; ++v) {
            if (bits) bits[(int64_t)f * n + v] = (uint8_t)neg(Lp[v]);
            if (post) post[(int64_t)f * n + v] = Lp[v];
        }
        free(c2v); free(v2c); free(Lp); free(mag);
    }
    free_colview(&cv);
    return 0;
}

/*
 * Unrolled normalized min-sum (T iterations, no early stop, no clamp) and its
 * reverse-mode derivative.
 *   forward: as orc_decode with algo = NMS and weights w[t][type];
 *   loss:    l = (1/(F n)) sum_{f,v} softplus( -(1 - 2 b_v) L_post,v(T) ),
 *            the binary cross-entropy of P(b = 1) = sigmoid(-L) against the true bits b.
 *   grads:   dl/dw [T][n_types]; optionally dl/dL_ch [F][n].
 * The derivative of |x| is taken as sign(x) with sign(0) = +1; the derivative
 * of the minimum over k != e goes to its lowest-index minimiser; sign products
 * are piecewise constant.  All intermediate messages are kept (a full tape).
 * prec32 != 0 runs the forward pass in binary32 as orc_decode does (so the
 * minimum and sign decisions are those of a binary32 decoder); the reverse
 * pass stays in double.
 */
int orc_nms_unrolled(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                     const uint8_t* edge_type, int32_t n_types,
                     int32_t F, const double* llr, const uint8_t* syn, const uint8_t* truth,
                     int32_t T, const double* weights, int32_t prec32,
                     double* loss_out, double* post_out, double* dw, double* dllr)
{
    if (n <= 0 || m < 0 || F < 0 || T < 1) return -1;
    const int64_t E = row_ptr[m];
    colview cv = make_colview(n, m, row_ptr, col_idx);
    const double inv_count = 1.0 / ((double)F * (double)n);
    /* per-frame partial results, summed in frame order afterwards so that the
     * result does not depend on the thread count */
    double* dw_frame = (double*)calloc((size_t)(F > 0 ? F : 1) * T * n_types, sizeof(double));
    double* loss_frame = (double*)calloc((size_t)(F > 0 ? F : 1), sizeof(double));

#pragma omp parallel
    {
        double* c2v = (double*)malloc((size_t)(T + 1) * (E > 0 ? E : 1) * sizeof(double)); /* c2v(t), t = 0..T */
        double* v2c = (double*)malloc((size_t)T * (E > 0 ? E : 1) * sizeof(double));       /* v2c(t), t = 0..T-1 */
        double* g_c2v = (double*)malloc((size_t)(E > 0 ? E : 1) * sizeof(double));
        double* g_v2c = (double*)malloc((size_t)(E > 0 ? E : 1) * sizeof(double));
        double* Lp = (double*)malloc((size_t)n * sizeof(double));
        double* gL = (double*)malloc((size_t)n * sizeof(double));

#pragma omp for schedule(dynamic, 1)
        for (int32_t f = 0; f < F; ++f) {
            const double* Lch = llr + (int64_t)f * n;
            const uint8_t* s = syn ? syn + (int64_t)f * m : NULL;
            const uint8_t* b = truth + (int64_t)f * n;
            double* dw_loc = dw_frame + (int64_t)f * T * n_types;
            double loss_loc = 0.0;
            for (int64_t e = 0; e < E; ++e) c2v[e] = 0.0;
            /* forward */
            for (int32_t t = 0; t < T; ++t) {
                const double* cin = c2v + (int64_t)t * E;
                double* vt = v2c + (int64_t)t * E;
                double* cout = c2v + (int64_t)(t + 1) * E;
                for (int32_t v = 0; v < n; ++v) {
                    double lp = rnd(1, Lch[v]);
                    if (prec32)
                        for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) lp = rnd(1, lp + cin[cv.edge[k]]);
                    for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) {
                        double a;
                        if (prec32) {
                            a = rnd(1, lp - cin[cv.edge[k]]);
                        } else {
                            a = Lch[v];
                            for (int32_t k2 = cv.ptr[v]; k2 < cv.ptr[v + 1]; ++k2)
                                if (k2 != k) a += cin[cv.edge[k2]];
                        }
                        vt[cv.edge[k]] = a;
                    }
                }
                for (int32_t c = 0; c < m; ++c) {
                    const double ssign = (s && (s[c] & 1)) ? -1.0 : 1.0;
                    for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
                        double sg = ssign, mn = INFINITY;
                        for (int32_t k = row_ptr[c]; k < row_ptr[c + 1]; ++k) {
                            if (k == e) continue;
                            if (neg(vt[k])) sg = -sg;
                            if (fabs(vt[k]) < mn) mn = fabs(vt[k]);
                        }
                        double w = weights[(int64_t)t * n_types + (edge_type ? edge_type[e] : 0)];
                        cout[e] = rnd(prec32, rnd(prec32, w) * (sg * mn));
                    }
                }
            }
            const double* cT = c2v + (int64_t)T * E;
            for (int32_t v = 0; v < n; ++v) {
                double a = rnd(prec32, Lch[v]);
                for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) a = rnd(prec32, a + cT[cv.edge[k]]);
                Lp[v] = a;
                if (post_out) post_out[(int64_t)f * n + v] = a;
                double z = -(1.0 - 2.0 * (b[v] & 1)) * a;           /* softplus(z) */
                double sp = z > 0 ? z + log1p(exp(-z)) : log1p(exp(z));
                loss_loc += sp * inv_count;
                double sig = z >= 0 ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z));
                gL[v] = -(1.0 - 2.0 * (b[v] & 1)) * sig * inv_count;
            }
            /* reverse: L_post(T) -> c2v(T) */
            for (int32_t v = 0; v < n; ++v)
                for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) g_c2v[cv.edge[k]] = gL[v];
            double* gch = dllr ? dllr + (int64_t)f * n : NULL;
            if (gch) for (int32_t v = 0; v < n; ++v) gch[v] = gL[v];
            for (int32_t t = T - 1; t >= 0; --t) {
                const double* vt = v2c + (int64_t)t * E;
                for (int64_t e = 0; e < E; ++e) g_v2c[e] = 0.0;
                /* through c2v(t+1) = w * sg_e * min_{k != e} |v2c_k| */
                for (int32_t c = 0; c < m; ++c) {
                    const double ssign = (s && (s[c] & 1)) ? -1.0 : 1.0;
                    for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
                        double sg = ssign, mn = INFINITY;
                        int32_t arg = -1;
                        for (int32_t k = row_ptr[c]; k < row_ptr[c + 1]; ++k) {
                            if (k == e) continue;
                            if (neg(vt[k])) sg = -sg;
                            if (fabs(vt[k]) < mn) { mn = fabs(vt[k]); arg = k; }
                        }
                        int32_t ty = edge_type ? edge_type[e] : 0;
                        double w = rnd(prec32, weights[(int64_t)t * n_types + ty]);
                        dw_loc[(int64_t)t * n_types + ty] += g_c2v[e] * sg * mn;
                        if (arg >= 0) {
                            double dabs = neg(vt[arg]) ? -1.0 : 1.0;
                            g_v2c[arg] += g_c2v[e] * w * sg * dabs;
                        }
                    }
                }
                /* through v2c(t)_e = L_ch + sum_{k != e} c2v(t)_k */
                for (int64_t e = 0; e < E; ++e) g_c2v[e] = 0.0;
                for (int32_t v = 0; v < n; ++v)
                    for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) {
                        double g = g_v2c[cv.edge[k]];
                        if (gch) gch[v] += g;
                        for (int32_t k2 = cv.ptr[v]; k2 < cv.ptr[v + 1]; ++k2)
                            if (k2 != k) g_c2v[cv.edge[k2]] += g;
                    }
                /* c2v(0) = 0 is a constant: nothing flows further at t = 0 */
            }
            loss_frame[f] = loss_loc;
        }
        free(c2v); free(v2c); free(g_c2v); free(g_v2c); free(Lp); free(gL);
    }
    double loss_total = 0.0;
    for (int64_t i = 0; i < (int64_t)T * n_types; ++i) dw[i] = 0.0;
    for (int32_t f = 0; f < F; ++f) {
        loss_total += loss_frame[f];
        for (int64_t i = 0; i < (int64_t)T * n_types; ++i) dw[i] += dw_frame[(int64_t)f * T * n_types + i];
    }
    if (loss_out) *loss_out = loss_total;
    free(dw_frame); free(loss_frame);
    free_colview(&cv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One check row of the check-node rule, shared by the step-wise functions  */
/* below (the same rule orc_decode writes out inline):                      */
/*   SP:  out_e = (1 - 2 s_c) prod_{k != e} sign(x_k) phi(sum_{k != e} phi(|x_k|)), */
/*        every x first clamped to [-clamp, clamp];                         */
/*   NMS: out_e = w_e (1 - 2 s_c) prod_{k != e} sign(x_k) min_{k != e} |x_k|. */
/* prec32 rounds every add, multiply and phi to binary32.                   */
/* ------------------------------------------------------------------------ */
static void check_row_rule(int32_t d, const double* x, double ssign, int32_t algo, int32_t prec32,
                           double clamp, const double* w, double* mag, double* out)
{
    for (int32_t k = 0; k < d; ++k) {
        double v = x[k];
        if (algo == ORC_SP) {
            if (v > clamp) v = clamp;
            if (v < -clamp) v = -clamp;
        }
        mag[k] = v;
    }
    for (int32_t e = 0; e < d; ++e) {
        double sg = ssign;
        for (int32_t k = 0; k < d; ++k)
            if (k != e && neg(mag[k])) sg = -sg;
        if (algo == ORC_SP) {
            double acc = 0.0;
            for (int32_t k = 0; k < d; ++k)
                if (k != e) acc = rnd(prec32, acc + rnd(prec32, phi(fabs(mag[k]))));
            out[e] = sg * rnd(prec32, phi(acc));
        } else {
            double mn = INFINITY;
            for (int32_t k = 0; k < d; ++k)
                if (k != e && fabs(mag[k]) < mn) mn = fabs(mag[k]);
            out[e] = rnd(prec32, rnd(prec32, w[e]) * (sg * mn));
        }
    }
}

/*
 * One flooding iteration from a given state, for step-by-step comparisons of
 * the two precisions: c2v_in = c2v(t) [E] (all zero at t = 0) -> c2v_out =
 * c2v(t+1) and post_out = L_post(t+1) [n], for one frame.  t selects the row
 * of weights.  The fp64 mode forms v2c_e = L_ch + sum_{c' != c} c2v_{c'}(t);
 * the binary32 mode first accumulates L_post(t) = L_ch + sum c2v(t) in
 * ascending check order in binary32 and forms v2c_e = L_post(t) - c2v_e(t),
 * which is what orc_decode does in each mode at iteration t.
 */
int orc_flood_step(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                   const uint8_t* edge_type, int32_t n_types, const double* llr, const uint8_t* s,
                   int32_t algo, int32_t t, int32_t store_half, int32_t prec32, double alpha,
                   const double* weights, double clamp, const double* c2v_in, double* c2v_out,
                   double* post_out)
{
    if (n <= 0 || m < 0 || t < 0) return -1;
    const int64_t E = row_ptr[m];
    colview cv = make_colview(n, m, row_ptr, col_idx);
    int32_t maxdeg = 1;
    for (int32_t c = 0; c < m; ++c)
        if (row_ptr[c + 1] - row_ptr[c] > maxdeg) maxdeg = row_ptr[c + 1] - row_ptr[c];
    double* v2c = (double*)malloc((size_t)(E > 0 ? E : 1) * sizeof(double));
    double* mag = (double*)malloc((size_t)maxdeg * sizeof(double));
    double* w = (double*)malloc((size_t)maxdeg * sizeof(double));
    double* out = (double*)malloc((size_t)maxdeg * sizeof(double));
    for (int32_t v = 0; v < n; ++v) {
        double lp = 0.0;
        if (prec32) {
            lp = rnd(1, llr[v]);
            for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) lp = rnd(1, lp + c2v_in[cv.edge[k]]);
        }
        for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) {
            double a;
            if (prec32) {
                a = rnd(1, lp - c2v_in[cv.edge[k]]);
            } else {
                a = llr[v];
                for (int32_t k2 = cv.ptr[v]; k2 < cv.ptr[v + 1]; ++k2)
                    if (k2 != k) a += c2v_in[cv.edge[k2]];
            }
            v2c[cv.edge[k]] = a;
        }
    }
    for (int32_t c = 0; c < m; ++c) {
        const int32_t e0 = row_ptr[c], d = row_ptr[c + 1] - e0;
        for (int32_t e = 0; e < d; ++e)
            w[e] = weights ? weights[(int64_t)t * n_types + (edge_type ? edge_type[e0 + e] : 0)] : alpha;
        check_row_rule(d, v2c + e0, (s && (s[c] & 1)) ? -1.0 : 1.0, algo, prec32, clamp, w, mag, out);
        for (int32_t e = 0; e < d; ++e) c2v_out[e0 + e] = store_half ? orc_round_half(out[e]) : out[e];
    }
    for (int32_t v = 0; v < n; ++v) {
        double a = rnd(prec32, llr[v]);
        for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) a = rnd(prec32, a + c2v_out[cv.edge[k]]);
        post_out[v] = a;
    }
    free(v2c); free(mag); free(w); free(out);
    free_colview(&cv);
    return 0;
}

/*
 * Layered (row-serial) belief propagation.  The paper names belief
 * propagation without a schedule (Sec. III-C); this is the serial schedule
 * over layers: rows are grouped into layers (layer l holds rows
 * layer_ptr[l] .. layer_ptr[l+1]-1, no two of which share a variable), and an
 * iteration updates the layers one after another, each from the messages its
 * predecessors in the same iteration have already replaced.
 *
 * fp64 mode (the definition): for every row c of layer l and edge e = (c, v),
 *     v2c_e = L_ch[v] + sum_{c' in N(v), c' != c} c2v_{c'}    (current values),
 *     c2v_e <- check rule of the row (as in orc_decode),
 * and after the last layer L_post[v] = L_ch[v] + sum_{c in N(v)} c2v_c.
 * Rows of one layer touch disjoint variables, so the order of rows inside a
 * layer does not matter.
 *
 * prec32 mode: the binary32 form a layered decoder runs.  It keeps the
 * posterior L[v] as a running value (L = L_ch rounded at the start) and, for
 * every edge of a row, forms x_e = L[v] - c2v_e(old), applies the check rule
 * and sets L[v] = x_e + c2v_e(new), each operation rounded to binary32.  In
 * exact arithmetic L[v] stays equal to L_ch[v] + sum c2v, so this is the fp64
 * mode up to rounding; it differs from it by the rounding of the running sum.
 *
 * Stopping, traces and outputs as orc_decode: the syndrome of the hard
 * decisions of L_post is tested before the first iteration and after each
 * (a check touching a NaN posterior counts as unsatisfied).  Returns -1 for
 * bad arguments, -2 when two rows of one layer share a variable.
 */
static int layers_disjoint(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                           int32_t n_layers, const int32_t* layer_ptr)
{
    int32_t* seen = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int32_t v = 0; v < n; ++v) seen[v] = -1;
    int ok = 1;
    for (int32_t l = 0; l < n_layers && ok; ++l)
        for (int32_t c = layer_ptr[l]; c < layer_ptr[l + 1] && ok; ++c)
            for (int32_t e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
                if (seen[col_idx[e]] == l) { ok = 0; break; }
                seen[col_idx[e]] = l;
            }
    free(seen);
    return ok;
}

/* One layered iteration (all layers) of one frame: c2v and L are updated in
 * place.  In fp64 mode L is recomputed from c2v at the end; in prec32 mode it
 * is the running posterior. */
static void layered_iteration(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                              const uint8_t* edge_type, int32_t n_types, const colview* cv,
                              int32_t n_layers, const int32_t* layer_ptr, const double* Lch,
                              const uint8_t* s, int32_t algo, int32_t t, int32_t store_half,
                              int32_t prec32, double alpha, const double* weights, double clamp,
                              double* c2v, double* L, double* x, double* mag, double* w, double* out)
{
    for (int32_t l = 0; l < n_layers; ++l) {
        for (int32_t c = layer_ptr[l]; c < layer_ptr[l + 1]; ++c) {
            const int32_t e0 = row_ptr[c], d = row_ptr[c + 1] - e0;
            for (int32_t e = 0; e < d; ++e) {
                const int32_t v = col_idx[e0 + e];
                if (prec32) {
                    x[e] = rnd(1, L[v] - c2v[e0 + e]);
                } else {
                    double a = Lch[v];
                    for (int32_t k = cv->ptr[v]; k < cv->ptr[v + 1]; ++k)
                        if (cv->edge[k] != e0 + e) a += c2v[cv->edge[k]];
                    x[e] = a;
                }
                w[e] = weights ? weights[(int64_t)t * n_types + (edge_type ? edge_type[e0 + e] : 0)] : alpha;
            }
            check_row_rule(d, x, (s && (s[c] & 1)) ? -1.0 : 1.0, algo, prec32, clamp, w, mag, out);
            for (int32_t e = 0; e < d; ++e) {
                c2v[e0 + e] = store_half ? orc_round_half(out[e]) : out[e];
                if (prec32) L[col_idx[e0 + e]] = rnd(1, x[e] + c2v[e0 + e]);
            }
        }
    }
    if (!prec32) {
        for (int32_t v = 0; v < n; ++v) {
            double a = Lch[v];
            for (int32_t k = cv->ptr[v]; k < cv->ptr[v + 1]; ++k) a += c2v[cv->edge[k]];
            L[v] = a;
        }
    }
}

int orc_decode_layered(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                       const uint8_t* edge_type, int32_t n_types, int32_t n_layers,
                       const int32_t* layer_ptr, int32_t F, const double* llr, const uint8_t* syn,
                       int32_t algo, int32_t T, int32_t early_stop, int32_t store_half, int32_t prec32,
                       double alpha, const double* weights, double clamp,
                       uint8_t* bits, double* post, int32_t* iters, uint8_t* ok,
                       double* trace, double* trace_scale, int32_t* trace_unsat)
{
    if (n <= 0 || m < 0 || F < 0 || T < 0 || n_layers < 0) return -1;
    if (layer_ptr[0] != 0 || layer_ptr[n_layers] != m) return -1;
    for (int32_t l = 0; l < n_layers; ++l)
        if (layer_ptr[l + 1] < layer_ptr[l]) return -1;
    if (!layers_disjoint(n, row_ptr, col_idx, n_layers, layer_ptr)) return -2;
    const int64_t E = row_ptr[m];
    colview cv = make_colview(n, m, row_ptr, col_idx);
    int32_t maxdeg = 1;
    for (int32_t c = 0; c < m; ++c)
        if (row_ptr[c + 1] - row_ptr[c] > maxdeg) maxdeg = row_ptr[c + 1] - row_ptr[c];

#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
        const double* Lch = llr + (int64_t)f * n;
        const uint8_t* s = syn ? syn + (int64_t)f * m : NULL;
        double* c2v = (double*)calloc((size_t)(E > 0 ? E : 1), sizeof(double));
        double* L = (double*)malloc((size_t)n * sizeof(double));
        double* x = (double*)malloc((size_t)maxdeg * sizeof(double));
        double* mag = (double*)malloc((size_t)maxdeg * sizeof(double));
        double* w = (double*)malloc((size_t)maxdeg * sizeof(double));
        double* out = (double*)malloc((size_t)maxdeg * sizeof(double));
        for (int32_t v = 0; v < n; ++v) L[v] = rnd(prec32, Lch[v]);
        int32_t t = 0;
        for (;;) {
            const int32_t u = count_unsat(m, row_ptr, col_idx, L, s);
            if (trace) memcpy(trace + ((int64_t)f * (T + 1) + t) * n, L, (size_t)n * sizeof(double));
            if (trace_scale) {
                double* sc = trace_scale + ((int64_t)f * (T + 1) + t) * n;
                for (int32_t v = 0; v < n; ++v) {
                    double a = fabs(Lch[v]);
                    for (int32_t k = cv.ptr[v]; k < cv.ptr[v + 1]; ++k) a += fabs(c2v[cv.edge[k]]);
                    sc[v] = a;
                }
            }
            if (trace_unsat) trace_unsat[(int64_t)f * (T + 1) + t] = u;
            if ((early_stop && u == 0) || t == T) {
                iters[f] = t;
                ok[f] = (uint8_t)(u == 0);
                break;
            }
            layered_iteration(n, row_ptr, col_idx, edge_type, n_types, &cv, n_layers, layer_ptr, Lch, s,
                              algo, t, store_half, prec32, alpha, weights, clamp, c2v, L, x, mag, w, out);
            ++t;
        }
        for (int32_t v = 0; v < n; ++v) {
            if (bits) bits[(int64_t)f * n + v] = (uint8_t)neg(L[v]);
            if (post) post[(int64_t)f * n + v] = L[v];
        }
        free(c2v); free(L); free(x); free(mag); free(w); free(out);
    }
    free_colview(&cv);
    return 0;
}

/*
 * One layered iteration of one frame from a given state (for step-by-step
 * comparisons): c2v [E] and post [n] are read and overwritten in place.  In
 * fp64 mode post is only written (the posterior is a function of c2v); in
 * prec32 mode post is the running binary32 posterior the iteration starts
 * from (L_ch rounded to binary32 before the first iteration).
 */
int orc_layered_step(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                     const uint8_t* edge_type, int32_t n_types, int32_t n_layers, const int32_t* layer_ptr,
                     const double* llr, const uint8_t* s, int32_t algo, int32_t t, int32_t store_half,
                     int32_t prec32, double alpha, const double* weights, double clamp,
                     double* c2v, double* post)
{
    if (n <= 0 || m < 0 || t < 0 || n_layers < 0) return -1;
    if (layer_ptr[0] != 0 || layer_ptr[n_layers] != m) return -1;
    if (!layers_disjoint(n, row_ptr, col_idx, n_layers, layer_ptr)) return -2;
    colview cv = make_colview(n, m, row_ptr, col_idx);
    int32_t maxdeg = 1;
    for (int32_t c = 0; c < m; ++c)
        if (row_ptr[c + 1] - row_ptr[c] > maxdeg) maxdeg = row_ptr[c + 1] - row_ptr[c];
    double* x = (double*)malloc((size_t)maxdeg * sizeof(double));
    double* mag = (double*)malloc((size_t)maxdeg * sizeof(double));
    double* w = (double*)malloc((size_t)maxdeg * sizeof(double));
    double* out = (double*)malloc((size_t)maxdeg * sizeof(double));
    layered_iteration(n, row_ptr, col_idx, edge_type, n_types, &cv, n_layers, layer_ptr, llr, s, algo, t,
                      store_half, prec32, alpha, weights, clamp, c2v, post, x, mag, w, out);
    free(x); free(mag); free(w); free(out);
    free_colview(&cv);
    return 0;
}
