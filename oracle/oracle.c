/*
 * FP64 CPU oracle for CountSketch / TensorSketch interpolative decomposition
 * (Malik & Becker, "Fast randomized matrix and tensor interpolative
 * decomposition using CountSketch").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * reference that the GPU library is checked against.  It shares no code, no
 * header and no table with the GPU library, and the GPU library never calls
 * it.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.
 *
 * Every routine is written as the definition it follows, in double precision,
 * with plain loops and a fixed summation order (increasing index).  No
 * blocking, no fusion, no reordering beyond what the definition states.
 *
 * Build: gcc -O2 -shared -fPIC -o _liboracle.so oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Counter-based hash stream (SplitMix64, Steele, Lea & Flood, OOPSLA 2014).
 * The paper only requires h(i) iid uniform on [L] and iid +-1 signs
 * (Section 1.3, CountSketch definition); the concrete generator is this
 * library's choice and is written here from the SplitMix64 publication:
 *   state_i = key + (i+1) * 0x9e3779b97f4a7c15
 *   z_i     = mix64(state_i)
 * mix64 is the published 64-bit finaliser (shift-xor-multiply, constants
 * 0xbf58476d1ce4e5b9 and 0x94d049bb133111eb, shifts 30/27/31).
 * The stream key for (seed, tag) is mix64(seed XOR mix64(tag)).
 * bucket = floor(hi32(z_i) * L / 2^32)    (Lemire's multiply-shift range map)
 * sign   = +1 if bit 0 of z_i is 0, else -1.
 * ---------------------------------------------------------------------- */
uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_stream_key(uint64_t seed, uint64_t tag) {
    return orc_mix64(seed ^ orc_mix64(tag));
}

/* z_i for i = 0..m-1 of the stream (seed, tag) */
void orc_stream(uint64_t seed, uint64_t tag, int64_t m, uint64_t* z) {
    uint64_t key = orc_stream_key(seed, tag);
    for (int64_t i = 0; i < m; ++i)
        z[i] = orc_mix64(key + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ULL);
}

/* The CountSketch maps h : [m] -> [L] and D = diag(+-1) (Section 1.3). */
void orc_hash(uint64_t seed, uint64_t tag, int64_t m, int64_t L,
              int32_t* bucket, int8_t* sign) {
    uint64_t key = orc_stream_key(seed, tag);
    for (int64_t i = 0; i < m; ++i) {
        uint64_t z = orc_mix64(key + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ULL);
        uint64_t hi = z >> 32;
        bucket[i] = (int32_t)((hi * (uint64_t)L) >> 32);
        sign[i] = (z & 1ULL) ? (int8_t)-1 : (int8_t)1;
    }
}

/* Modified hash of Remark 2 / Proposition 4: h~(i) = f(pi(i)) with
 * f(q) = q for q < L and f(q) = x[q] (iid uniform on [L]) otherwise.
 * 0-based: pi is a permutation of 0..m-1, x[q] in [0, L). */
void orc_fullrank_hash(int64_t m, int64_t L, const int64_t* pi, const int32_t* x,
                       int32_t* bucket) {
    for (int64_t i = 0; i < m; ++i) {
        int64_t q = pi[i];
        bucket[i] = (q < L) ? (int32_t)q : x[q];
    }
}

/* ------------------------------------------------------------------------
 * CountSketch Y = S A = Phi D A (Section 1.3; Algorithm 2, step "compute
 * sketch"): every row i of A, multiplied by its sign, is added into row
 * h(i) of Y.  Rows are visited in increasing i.
 * A is m x n row-major with leading dimension lda; Y is L x n row-major.
 * ---------------------------------------------------------------------- */
void orc_countsketch_dense(int64_t m, int64_t n, const double* A, int64_t lda,
                           const int32_t* bucket, const int8_t* sign, int64_t L,
                           double* Y) {
    memset(Y, 0, sizeof(double) * (size_t)(L * n));
    for (int64_t i = 0; i < m; ++i) {
        double s = (double)sign[i];
        double* y = Y + (int64_t)bucket[i] * n;
        const double* a = A + i * lda;
        for (int64_t j = 0; j < n; ++j) y[j] += s * a[j];
    }
}

/* Same definition for A in CSR form: only the stored entries are added;
 * duplicate (row, col) entries are summed. */
void orc_countsketch_csr(int64_t m, int64_t n, const int64_t* rowptr,
                         const int32_t* colind, const double* val,
                         const int32_t* bucket, const int8_t* sign, int64_t L,
                         double* Y) {
    memset(Y, 0, sizeof(double) * (size_t)(L * n));
    for (int64_t i = 0; i < m; ++i) {
        double s = (double)sign[i];
        double* y = Y + (int64_t)bucket[i] * n;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) y[colind[e]] += s * val[e];
    }
}

/* Plain product C = G B, G l x q, B q x n, all row-major: the second-stage
 * Gaussian projection of the sketch (Section 1.2.1, Gaussian sketch). */
void orc_gemm(int64_t l, int64_t q, int64_t n, const double* G, const double* B,
              double* C) {
    for (int64_t i = 0; i < l; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t p = 0; p < q; ++p) acc += G[i * q + p] * B[p * n + j];
            C[i * n + j] = acc;
        }
}

/* ------------------------------------------------------------------------
 * Matrix ID via rank-K column-pivoted QR (Algorithm 1, with column-pivoted
 * QR in place of strong RRQR as the paper does in practice, Section 1.2.1).
 *
 * Input Y: l x n row-major.  For t = 0..k-1:
 *   nu_j = sum_{i>=t} Y[i][j]^2 for every column j not yet chosen
 *          (recomputed from scratch every step, no downdating);
 *   pivot = argmax nu_j, ties to the smallest column index;
 *   if nu_pivot == 0 stop (rank deficient: k_eff = t);
 *   Householder reflector H = I - tau v v^T of the pivot column's rows t..l-1
 *   (LAPACK dlarfg convention: v[0] = 1, beta = -sign(alpha) * norm), applied
 *   to every column not yet chosen; R[t][pivot] = beta, R[t][j] = Y[i=t][j].
 * Then T = R11^{-1} R12 by back-substitution (Algorithm 1, last step) and
 * P = [I T] Pi^T written in the original column order: P[:, J[t]] = e_t and
 * P[:, j] = R11^{-1} R[0:k, j] for every other column j.
 *
 * Outputs: J[k] (0-based), P (k x n row-major, rows >= k_eff left zero),
 * optional Rtop (k x n row-major: row t of R in original column order),
 * optional nu_trace (k x n: nu at the start of step t, -1 for chosen columns).
 * Returns k_eff.
 * ---------------------------------------------------------------------- */
int64_t orc_cpqr_id(int64_t l, int64_t n, int64_t k, const double* Y,
                    int64_t* J, double* P, double* Rtop, double* nu_trace) {
    /* column-major working copy: W[j*l + i] = Y[i][j] (layout only) */
    double* W = (double*)malloc(sizeof(double) * (size_t)(l * n));
    char* chosen = (char*)calloc((size_t)n, 1);
    double* R = (double*)calloc((size_t)(k * n), sizeof(double));
    double* v = (double*)malloc(sizeof(double) * (size_t)l);
    for (int64_t i = 0; i < l; ++i)
        for (int64_t j = 0; j < n; ++j) W[j * l + i] = Y[i * n + j];

    int64_t keff = k;
    for (int64_t t = 0; t < k; ++t) {
        int64_t piv = -1;
        double best = -1.0;
        for (int64_t j = 0; j < n; ++j) {
            if (chosen[j]) {
                if (nu_trace) nu_trace[t * n + j] = -1.0;
                continue;
            }
            double s = 0.0;
            for (int64_t i = t; i < l; ++i) s += W[j * l + i] * W[j * l + i];
            if (nu_trace) nu_trace[t * n + j] = s;
            if (s > best) { best = s; piv = j; }
        }
        if (piv < 0 || best == 0.0) { keff = t; break; }
        J[t] = piv;
        chosen[piv] = 1;

        /* Householder reflector of x = W[piv][t..l-1] */
        const double* x = W + piv * l;
        double alpha = x[t];
        double sig2 = 0.0;
        for (int64_t i = t + 1; i < l; ++i) sig2 += x[i] * x[i];
        double tau, beta;
        if (sig2 == 0.0) {
            tau = 0.0;
            beta = alpha;
            for (int64_t i = t; i < l; ++i) v[i] = 0.0;
            v[t] = 1.0;
        } else {
            double nrm = sqrt(alpha * alpha + sig2);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            double scal = 1.0 / (alpha - beta);
            v[t] = 1.0;
            for (int64_t i = t + 1; i < l; ++i) v[i] = x[i] * scal;
        }
        R[t * n + piv] = beta;
        /* apply H to the pivot column too, so W stays consistent */
        for (int64_t j = 0; j < n; ++j) {
            if (chosen[j] && j != piv) continue;
            double* w = W + j * l;
            double d = 0.0;
            for (int64_t i = t; i < l; ++i) d += v[i] * w[i];
            d *= tau;
            for (int64_t i = t; i < l; ++i) w[i] -= d * v[i];
            if (j != piv) R[t * n + j] = w[t];
        }
    }

    /* R11 entries: R11[a][b] = R[a][J[b]] for a <= b (upper triangular). */
    memset(P, 0, sizeof(double) * (size_t)(k * n));
    double* b = (double*)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int64_t j = 0; j < n; ++j) {
        if (chosen[j]) continue;
        /* back-substitution: solve R11 x = R[0:keff, j] */
        for (int64_t a = keff - 1; a >= 0; --a) {
            double s = R[a * n + j];
            for (int64_t c = a + 1; c < keff; ++c) s -= R[a * n + J[c]] * b[c];
            b[a] = s / R[a * n + J[a]];
        }
        for (int64_t a = 0; a < keff; ++a) P[a * n + j] = b[a];
    }
    for (int64_t a = 0; a < keff; ++a) P[a * n + J[a]] = 1.0;
    for (int64_t a = keff; a < k; ++a) J[a] = -1;
    if (Rtop) memcpy(Rtop, R, sizeof(double) * (size_t)(k * n));

    free(b); free(v); free(R); free(chosen); free(W);
    return keff;
}

/* ------------------------------------------------------------------------
 * TensorSketch of M = (Khatri-Rao of the factor matrices) diag(lambda)
 * (eq. for M; TensorSketch definition with H and S, Section 1.3).
 * Column r of T M is lambda_r * (c_1 (*) c_2 (*) ... (*) c_N), where
 * c_n = S^(n) a^(n)_r is the mode-n CountSketch of column r of factor n and
 * (*) is circular convolution of length Jlen.  The convolution is evaluated
 * directly from its definition, y[(u+v) mod Jlen] += c[u] * d[v], which is the
 * sum over all index tuples of S(i) * M[i, r] into bucket H(i), with no FFT.
 *
 * factors[n] is I_n x R column-major with leading dimension ld[n]
 * (entry (i, r) at factors[n][r*ld[n] + i]).  bucket[n], sign[n] are the
 * per-mode maps h_n, s_n.  cols lists the ncols columns to sketch (NULL: all
 * R).  Output Y is Jlen x ncols column-major: Y[c*Jlen + b].
 * ---------------------------------------------------------------------- */
void orc_tensorsketch(int32_t N, const int64_t* dims, const int64_t* ld, int64_t R,
                      const double* const* factors, const double* lambda,
                      const int32_t* const* bucket, const int8_t* const* sign,
                      int64_t Jlen, const int64_t* cols, int64_t ncols, double* Y) {
    double* acc = (double*)malloc(sizeof(double) * (size_t)Jlen);
    double* c = (double*)malloc(sizeof(double) * (size_t)Jlen);
    double* nxt = (double*)malloc(sizeof(double) * (size_t)Jlen);
    if (!cols) ncols = R;
    for (int64_t q = 0; q < ncols; ++q) {
        int64_t r = cols ? cols[q] : q;
        for (int32_t md = 0; md < N; ++md) {
            memset(c, 0, sizeof(double) * (size_t)Jlen);
            const double* a = factors[md] + r * ld[md];
            for (int64_t i = 0; i < dims[md]; ++i)
                c[bucket[md][i]] += (double)sign[md][i] * a[i];
            if (md == 0) {
                memcpy(acc, c, sizeof(double) * (size_t)Jlen);
            } else {
                memset(nxt, 0, sizeof(double) * (size_t)Jlen);
                for (int64_t u = 0; u < Jlen; ++u) {
                    if (acc[u] == 0.0) continue;
                    for (int64_t w = 0; w < Jlen; ++w) {
                        int64_t b = u + w;
                        if (b >= Jlen) b -= Jlen;
                        nxt[b] += acc[u] * c[w];
                    }
                }
                memcpy(acc, nxt, sizeof(double) * (size_t)Jlen);
            }
        }
        for (int64_t b = 0; b < Jlen; ++b) Y[q * Jlen + b] = lambda[r] * acc[b];
    }
    free(nxt); free(c); free(acc);
}

/* New s-values of the kept terms (Algorithm 3, s-value step):
 * lambda_hat[t] = lambda[J[t]] * sum_r P[t][r], r in increasing order. */
void orc_lambda_hat(int64_t k, int64_t n, const double* P, const int64_t* J,
                    const double* lambda, double* lhat) {
    for (int64_t t = 0; t < k; ++t) {
        double s = 0.0;
        for (int64_t r = 0; r < n; ++r) s += P[t * n + r];
        lhat[t] = lambda[J[t]] * s;
    }
}

/* Gaussian matrix entries drawn from the stream (seed, tag | 2^63): entry e
 * (row-major) takes outputs 2e and 2e+1 of the stream as uniforms
 * u1 = ((z >> 11) + 1) 2^-53 in (0, 1] and u2 = (z >> 11) 2^-53 in [0, 1),
 * and the Box-Muller transform g = sqrt(-2 ln u1) cos(2 pi u2)
 * (Box & Muller 1958) gives an N(0, 1) value. */
void orc_gaussian(uint64_t seed, uint64_t tag, int64_t count, double* g) {
    const uint64_t key = orc_stream_key(seed, tag | (1ULL << 63));
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t e = 0; e < count; ++e) {
        const uint64_t z1 = orc_mix64(key + (uint64_t)(2 * e + 1) * 0x9e3779b97f4a7c15ULL);
        const uint64_t z2 = orc_mix64(key + (uint64_t)(2 * e + 2) * 0x9e3779b97f4a7c15ULL);
        const double u1 = (double)((z1 >> 11) + 1) * 0x1p-53;
        const double u2 = (double)(z2 >> 11) * 0x1p-53;
        g[e] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    }
}
