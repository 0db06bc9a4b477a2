/*
 * sanitize_check.c -- driver for a sanitizer build of the FP64 oracle (test infrastructure).
 *
 * Built with gcc -fsanitize=address,undefined together with reann_oracle.c by
 * tests/test_oracle_sanitizers.py; runs every exported entry point of the oracle (neighbour
 * export, whole-system, decomposed, naive-decomposition and extended-halo evaluations, with
 * forces, virial and the per-layer debug outputs) on a small periodic box whose side is shorter
 * than twice the list cutoff (so many periodic images appear), then checks that the decomposed
 * and halo results equal the whole-system one; then the same whole and decomposed evaluations of
 * the radial message form.  Exits non-zero on any failure; the sanitizers
 * abort on any memory or undefined-behaviour error.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_species, L, K, T_max, n_hidden, hidden;
    double r_c, ang_scale, energy_scale;
    const double *centres, *alphas, *c0, *msg, *en;
    int32_t form;
} model_t;

int64_t oracle_neighbors(int64_t n, const double *pos, const double *cell, const int32_t *pbc, double rcut,
                         const int32_t *decomp, int64_t *row, int64_t *jout, int32_t *sout);
int oracle_eval(const model_t *m, int64_t n, const double *pos, const int32_t *species, const double *cell,
                const int32_t *pbc, double skin, int32_t T, const int32_t *decomp, int32_t naive, int32_t n_threads,
                double *energy, double *atom_energy, double *forces, double *virial, double *S_out, double *c_out);
int oracle_eval_halo(const model_t *m, int64_t n, const double *pos, const int32_t *species, const double *cell,
                     const int32_t *pbc, double skin, int32_t T, const int32_t *decomp, int32_t n_threads,
                     double *energy, double *atom_energy, double *forces, double *virial, int64_t *work);

static uint64_t lcg = 12345;
static double urand(void) {   /* uniform in [0, 1) from a 64-bit linear congruential generator */
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

int main(void) {
    enum { N = 20, NS = 2, L = 2, K = 4, TM = 3, NH = 1, HID = 8 };
    const int NL = 10, F = (L + 1) * K * (K + 1) / 2;
    double pos[3 * N], cell[9] = { 7.3, 0, 0, 0, 6.9, 0, 0, 0, 7.1 };
    int32_t spec[N], pbc[3] = { 1, 1, 1 };
    for (int i = 0; i < N; ++i) {   /* points at least 1.2 A apart */
        for (;;) {
            double p[3] = { urand() * 7.3, urand() * 6.9, urand() * 7.1 };
            int ok = 1;
            for (int j = 0; j < i && ok; ++j) {
                double d2 = 0;
                for (int a = 0; a < 3; ++a) {
                    double d = p[a] - pos[3 * j + a];
                    double L_ = cell[4 * a];
                    d -= L_ * floor(d / L_ + 0.5);
                    d2 += d * d;
                }
                ok = d2 > 1.44;
            }
            if (ok) { memcpy(pos + 3 * i, p, sizeof p); break; }
        }
        spec[i] = i % NS;
    }
    double centres[K], alphas[K], c0[NS * K];
    for (int k = 0; k < K; ++k) { centres[k] = 4.0 * k / (K - 1); alphas[k] = 2.0; }
    for (int k = 0; k < NS * K; ++k) c0[k] = urand() - 0.5;
    const int nn_msg = HID * F + HID + K * HID + K, nn_en = HID * F + HID + HID + 1;
    double *msg = malloc(sizeof(double) * (TM - 1) * NS * nn_msg), *en = malloc(sizeof(double) * NS * nn_en);
    for (int k = 0; k < (TM - 1) * NS * nn_msg; ++k) msg[k] = (urand() - 0.5) * 0.6;
    for (int k = 0; k < NS * nn_en; ++k) en[k] = (urand() - 0.5) * 0.6;
    model_t m = { NS, L, K, TM, NH, HID, 4.0, 0.25, 1.0, centres, alphas, c0, msg, en, 0 };
    const double skin = 0.5;
    int32_t whole[3] = { 1, 1, 1 }, split[3] = { 2, 1, 2 };

    int64_t cnt = oracle_neighbors(N, pos, cell, pbc, m.r_c + skin, split, NULL, NULL, NULL);
    if (cnt <= 0) { fprintf(stderr, "neighbour count %lld\n", (long long)cnt); return 1; }
    int64_t *row = malloc(sizeof(int64_t) * (N + 1)), *jj = malloc(sizeof(int64_t) * cnt);
    int32_t *sh = malloc(sizeof(int32_t) * 3 * cnt);
    if (oracle_neighbors(N, pos, cell, pbc, m.r_c + skin, split, row, jj, sh) != cnt) return 1;

    double E0, Ei[N], F0[3 * N], W0[9], S[TM * N * NL * K], c[TM * N * K];
    if (oracle_eval(&m, N, pos, spec, cell, pbc, skin, TM, whole, 0, 2, &E0, Ei, F0, W0, S, c)) return 1;
    double E1, F1[3 * N], W1[9], E2, E3, F3[3 * N], W3[9];
    int64_t work[2 * TM];
    if (oracle_eval(&m, N, pos, spec, cell, pbc, skin, TM, split, 0, 2, &E1, NULL, F1, W1, NULL, NULL)) return 1;
    if (oracle_eval(&m, N, pos, spec, cell, pbc, skin, TM, split, 1, 2, &E2, NULL, NULL, NULL, NULL, NULL)) return 1;
    if (oracle_eval_halo(&m, N, pos, spec, cell, pbc, skin, TM, split, 2, &E3, NULL, F3, W3, work)) return 1;
    double fmax = 0, dF1 = 0, dF3 = 0;
    for (int k = 0; k < 3 * N; ++k) {
        fmax = fmax > fabs(F0[k]) ? fmax : fabs(F0[k]);
        dF1 = fmax > 0 && fabs(F1[k] - F0[k]) > dF1 ? fabs(F1[k] - F0[k]) : dF1;
        dF3 = fabs(F3[k] - F0[k]) > dF3 ? fabs(F3[k] - F0[k]) : dF3;
    }
    printf("pairs %lld  E whole %.12f  split %.12f  naive %.12f  halo %.12f  max|dF| %.2e %.2e\n", (long long)cnt,
           E0, E1, E2, E3, dF1, dF3);
    int bad = fabs(E1 - E0) > 1e-10 * fabs(E0) || fabs(E3 - E0) > 1e-10 * fabs(E0) || dF1 > 1e-9 * fmax ||
              dF3 > 1e-9 * fmax;

    /* the radial form: L = 0, F = K features, residual updates */
    const int FR = K, rn_msg = HID * FR + HID + K * HID + K, rn_en = HID * FR + HID + HID + 1;
    model_t mr = { NS, 0, K, TM, NH, HID, 4.0, 0.25, 1.0, centres, alphas, c0, msg, en, 1 };
    (void)rn_msg; (void)rn_en;   /* smaller than the REANN blobs above, which they reuse */
    double Er0, Eri[N], Fr0[3 * N], Wr0[9], Sr[TM * N * K], cr[TM * N * K], Er1, Fr1[3 * N], Wr1[9], Er2;
    if (oracle_eval(&mr, N, pos, spec, cell, pbc, skin, TM, whole, 0, 2, &Er0, Eri, Fr0, Wr0, Sr, cr)) return 1;
    if (oracle_eval(&mr, N, pos, spec, cell, pbc, skin, TM, split, 0, 2, &Er1, NULL, Fr1, Wr1, NULL, NULL)) return 1;
    if (oracle_eval(&mr, N, pos, spec, cell, pbc, skin, TM, split, 1, 2, &Er2, NULL, NULL, NULL, NULL, NULL)) return 1;
    double frmax = 0, dFr = 0;
    for (int k = 0; k < 3 * N; ++k) {
        frmax = frmax > fabs(Fr0[k]) ? frmax : fabs(Fr0[k]);
        dFr = fabs(Fr1[k] - Fr0[k]) > dFr ? fabs(Fr1[k] - Fr0[k]) : dFr;
    }
    printf("radial form: E whole %.12f  split %.12f  naive %.12f  max|dF| %.2e\n", Er0, Er1, Er2, dFr);
    bad = bad || fabs(Er1 - Er0) > 1e-10 * fabs(Er0) || dFr > 1e-9 * frmax;
    free(msg); free(en); free(row); free(jj); free(sh);
    return bad ? 2 : 0;
}
