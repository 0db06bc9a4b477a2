/*
 * reann_oracle.c -- plain, slow FP64 CPU oracle for the REANN message-passing
 * energy, forces and virial, evaluated either for the whole periodic system or
 * split into spatial subdomains that exchange ghost-atom messages once per
 * message-passing (MP) layer.
 *
 * TEST INFRASTRUCTURE ONLY.  It exists to check the GPU library; only the test
 * suite, the package's smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code, header or table with the GPU path.
 *
 * What it follows (Xia & Jiang, "Efficient Parallelization of Message Passing
 * Neural Networks"):
 *   Sec. 2.1, Eq. (1)  embedded atom density of atom i from orbital sums over the
 *                      neighbours j inside r_c, squared with the l!/(lx!ly!lz!) weights
 *   Sec. 2.1           primitive Gaussian-type orbitals with centre, width and
 *                      angular momenta (lx,ly,lz), l <= L; element-wise coefficient c_j;
 *                      N_phi(N_phi+1)(L+1)/2 features
 *   Sec. 2.1, Eq. (2)  message update c_i^t = M^{t-1}_{s_i}(rho_i^{t-1}), 1 <= t <= T-1
 *   Sec. 2.1           atomic energies from the last atomic NN; E = sum_i E_i; T=1 is EANN
 *   Sec. 2.2           one neighbour list reused by all layers; spatial decomposition
 *                      into local atoms (LAs) and ghost atoms (GAs); GA messages copied
 *                      from their owners in every layer
 *   Sec. 2.2, Eqs. (3)-(5)  forces by the chain rule through rho, c and G; VJPs of
 *                      GA messages (dE/dc) and GA forces reduced onto their owners;
 *                      dc^0/dr = 0
 *
 * Readings where the paper is silent (each one also stated where it is used):
 *   R1 features: rho[l,(a,b)] = sum_{|lambda|=l} l!/lambda! S[lambda,a] S[lambda,b] for
 *      a <= b, which gives the stated (L+1)K(K+1)/2 count; order l, then a, then b >= a.
 *   R2 c_j is a K-vector multiplying primitive m element-wise; c^0 is a per-element vector.
 *   R3 cutoff f_c(r) = (cos(pi r / r_c)/2 + 1/2)^2 for r < r_c, else 0.
 *   R4 radial R_m(r) = exp(-alpha_m (r - r_m)^2); angular A_lambda(d) = prod (s d_x)^lx ...
 *      with s = ang_scale, d = x_j - x_i.
 *   R5 atomic NN: hidden layers Linear+SiLU, linear output; one NN per (layer, element);
 *      E_i = energy_scale * NN^E_{s_i}(rho_i^{T-1}).
 *   R6 virial W = sum over directed edges d (x) f with f = -dE/dd, in eV.
 *   R7 neighbours: every copy (j, n) of atom j shifted by n lattice vectors, (j,n) != (i,0),
 *      with d2 = fma(dz,dz, fma(dy,dy, dx*dx)) < (r_c+skin)^2 in FP64; only r < r_c contributes.
 *   R8 wrap w = x - floor(x/L)*L, then +L if negative, then -L if >= L, each step rounded.
 *   R9 subdomain k of P along an axis is [k*h, (k+1)*h) with h = L/P (the last ends at L);
 *      ghosts of a subdomain are all copies (j,n) other than its own locals whose position
 *      lies within shell = r_c + skin + 1e-6 A of the subdomain box on every split or
 *      periodic axis.  Non-periodic axes are not split (P = 1) and not wrapped.
 *   R14 a second message form on the same exchange (Sec. 2.2, the paragraph on other
 *      MPNNs that aggregate messages over neighbours, invariant ones such as SchNet among
 *      them): the "radial" form takes L = 0 and uses the orbital sum itself as the K
 *      features, x_i[m] = S_i[0][m] = sum_j c_j[m] R_m(r_ij) f_c(r_ij) (linear in the
 *      neighbours' messages, a per-channel Gaussian filter), and updates messages with a
 *      residual, c_i^{t+1} = c_i^t + M^t_{s_i}(x_i^t); E_i = energy_scale * NN^E_{s_i}(x_i^{T-1}).
 *      Its adjoint carries dE/dc^{t+1} into dE/dc^t through the residual.
 *   R15 the literal reading of Eq. (1) (the "diag" form): only the squares,
 *      rho[l,a] = sum_{|lambda|=l} l!/lambda! S[lambda,a]^2, F = (L+1) K; everything else as R1-R5.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no contraction anywhere, so the
 * neighbour predicate is exactly the expression above).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OM_OK 0
#define OM_EINVAL (-1)
#define OM_ENOMEM (-3)

#define OM_FORM_REANN 0
#define OM_FORM_RADIAL 1   /* reading R14 */
#define OM_FORM_DIAG 2     /* reading R15 */

typedef struct {
    int32_t n_species, L, K, T_max, n_hidden, hidden;
    double r_c, ang_scale, energy_scale;
    const double *centres; /* [K] */
    const double *alphas;  /* [K] */
    const double *c0;      /* [n_species][K] */
    const double *msg;     /* message NNs, see om_mlp_offset */
    const double *en;      /* energy NNs */
    int32_t form;          /* OM_FORM_REANN (Eqs. (1)-(2)) or OM_FORM_RADIAL (reading R14) */
} om_model;

/* ---------------------------------------------------------------- helpers -- */

static int om_nlambda(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
static int om_nfeat(int L, int K) { return (L + 1) * K * (K + 1) / 2; }
/* features per atom: the paired density of Eq. (1), or the K orbital sums of the radial form */
static int om_model_nfeat(const om_model *m) {
    if (m->form == OM_FORM_RADIAL) return m->K;
    if (m->form == OM_FORM_DIAG) return (m->L + 1) * m->K;
    return om_nfeat(m->L, m->K);
}

static double om_fact(int n) { double f = 1.0; for (int k = 2; k <= n; ++k) f *= k; return f; }

/* Cartesian components lambda = (lx,ly,lz), l = lx+ly+lz <= L, listed by l, then
   lx descending, then ly descending; with their l and multinomial weight l!/lambda!. */
typedef struct { int n; int lx[64], ly[64], lz[64], l[64]; double w[64]; } om_lambda;

static void om_lambda_init(int L, om_lambda *q) {
    int k = 0;
    for (int l = 0; l <= L; ++l)
        for (int lx = l; lx >= 0; --lx)
            for (int ly = l - lx; ly >= 0; --ly) {
                int lz = l - lx - ly;
                q->lx[k] = lx; q->ly[k] = ly; q->lz[k] = lz; q->l[k] = l;
                q->w[k] = om_fact(l) / (om_fact(lx) * om_fact(ly) * om_fact(lz));
                ++k;
            }
    q->n = k;
}

/* Parameter count of an atomic NN with dims [d0, d1 x nh, dout]. */
static int64_t om_mlp_size(int F, int H, int nh, int dout) {
    int64_t n = 0; int prev = F;
    for (int k = 0; k < nh; ++k) { n += (int64_t)H * prev + H; prev = H; }
    n += (int64_t)dout * prev + dout;
    return n;
}

static const double *om_msg_params(const om_model *m, int t, int s) {
    int F = om_model_nfeat(m);
    return m->msg + ((int64_t)t * m->n_species + s) * om_mlp_size(F, m->hidden, m->n_hidden, m->K);
}

static const double *om_en_params(const om_model *m, int s) {
    int F = om_model_nfeat(m);
    return m->en + (int64_t)s * om_mlp_size(F, m->hidden, m->n_hidden, 1);
}

static double om_silu(double z) { return z / (1.0 + exp(-z)); }
static double om_dsilu(double z) { double sg = 1.0 / (1.0 + exp(-z)); return sg * (1.0 + z * (1.0 - sg)); }

/* Atomic NN forward: x[F] -> y[dout].  Hidden layers z = W h + b, h = silu(z);
   output y = W h + b (reading R5).  W is row-major [out][in]. */
static void om_mlp_forward(const double *p, int F, int H, int nh, int dout, const double *x, double *y) {
    double a[1024], b[1024];
    const double *in = x; int din = F;
    for (int k = 0; k < nh; ++k) {
        const double *W = p; p += (int64_t)H * din;
        const double *bb = p; p += H;
        for (int o = 0; o < H; ++o) {
            double z = bb[o];
            for (int q = 0; q < din; ++q) z += W[(int64_t)o * din + q] * in[q];
            a[o] = om_silu(z);
        }
        memcpy(b, a, sizeof(double) * H); in = b; din = H;
    }
    const double *W = p; p += (int64_t)dout * din;
    const double *bb = p;
    for (int o = 0; o < dout; ++o) {
        double z = bb[o];
        for (int q = 0; q < din; ++q) z += W[(int64_t)o * din + q] * in[q];
        y[o] = z;
    }
}

/* Vector-Jacobian product of the atomic NN: given x and ybar = dE/dy, return
   xbar = (dy/dx)^T ybar.  The forward activations are recomputed here. */
static void om_mlp_vjp(const double *p, int F, int H, int nh, int dout, const double *x,
                       const double *ybar, double *xbar) {
    enum { MAXL = 8 };
    double z[MAXL][1024], h[MAXL][1024];
    const double *Wk[MAXL + 1];
    int din = F; const double *in = x;
    for (int k = 0; k < nh; ++k) {
        Wk[k] = p; const double *bb = p + (int64_t)H * din; p = bb + H;
        for (int o = 0; o < H; ++o) {
            double zz = bb[o];
            for (int q = 0; q < din; ++q) zz += Wk[k][(int64_t)o * din + q] * in[q];
            z[k][o] = zz; h[k][o] = om_silu(zz);
        }
        in = h[k]; din = H;
    }
    Wk[nh] = p;
    /* hbar of the last hidden layer = W_out^T ybar */
    double g[1024], gz[1024];
    int dprev = nh > 0 ? H : F;
    for (int q = 0; q < dprev; ++q) {
        double s = 0.0;
        for (int o = 0; o < dout; ++o) s += Wk[nh][(int64_t)o * dprev + q] * ybar[o];
        g[q] = s;
    }
    for (int k = nh - 1; k >= 0; --k) {
        for (int o = 0; o < H; ++o) gz[o] = g[o] * om_dsilu(z[k][o]);
        int dk = (k == 0) ? F : H;
        for (int q = 0; q < dk; ++q) {
            double s = 0.0;
            for (int o = 0; o < H; ++o) s += Wk[k][(int64_t)o * dk + q] * gz[o];
            g[q] = s;
        }
    }
    memcpy(xbar, g, sizeof(double) * F);
}

/* Density features from orbital sums S[lambda][m] (Eq. (1), reading R1). */
static void om_density(const om_lambda *q, int L, int K, const double *S, double *rho) {
    int f = 0;
    for (int l = 0; l <= L; ++l)
        for (int a = 0; a < K; ++a)
            for (int b = a; b < K; ++b) {
                double s = 0.0;
                for (int k = 0; k < q->n; ++k)
                    if (q->l[k] == l) s += q->w[k] * S[k * K + a] * S[k * K + b];
                rho[f++] = s;
            }
}

/* Adjoint of om_density: Sbar[lambda][a] = d(sum_f rhobar_f rho_f)/dS[lambda][a]. */
static void om_density_vjp(const om_lambda *q, int L, int K, const double *S, const double *rhobar,
                           double *Sbar) {
    int nl = q->n;
    memset(Sbar, 0, sizeof(double) * nl * K);
    int f = 0;
    for (int l = 0; l <= L; ++l)
        for (int a = 0; a < K; ++a)
            for (int b = a; b < K; ++b) {
                double rb = rhobar[f++];
                for (int k = 0; k < nl; ++k) {
                    if (q->l[k] != l) continue;
                    Sbar[k * K + a] += rb * q->w[k] * S[k * K + b];
                    Sbar[k * K + b] += rb * q->w[k] * S[k * K + a];
                }
            }
}

/* The NN input of an atom from its orbital sums: the density of Eq. (1), or for the radial
   form (reading R14) the K sums of lambda = 0 themselves; and the adjoint of that map. */
static void om_features(const om_model *m, const om_lambda *q, const double *S, double *rho) {
    const int K = m->K;
    if (m->form == OM_FORM_RADIAL) { memcpy(rho, S, sizeof(double) * K); return; }
    if (m->form == OM_FORM_DIAG) {   /* reading R15: the squares of Eq. (1) */
        for (int l = 0; l <= m->L; ++l)
            for (int a = 0; a < K; ++a) {
                double s = 0.0;
                for (int k = 0; k < q->n; ++k)
                    if (q->l[k] == l) s += q->w[k] * S[k * K + a] * S[k * K + a];
                rho[l * K + a] = s;
            }
        return;
    }
    om_density(q, m->L, K, S, rho);
}
static void om_features_vjp(const om_model *m, const om_lambda *q, const double *S, const double *rhobar,
                            double *Sbar) {
    const int K = m->K;
    if (m->form == OM_FORM_RADIAL) { memcpy(Sbar, rhobar, sizeof(double) * K); return; }
    if (m->form == OM_FORM_DIAG) {
        for (int k = 0; k < q->n; ++k)
            for (int a = 0; a < K; ++a) Sbar[k * K + a] = 2.0 * q->w[k] * S[k * K + a] * rhobar[q->l[k] * K + a];
        return;
    }
    om_density_vjp(q, m->L, K, S, rhobar, Sbar);
}

/* Cutoff (reading R3) and its derivative. */
static double om_fc(double r, double rc) {
    if (r >= rc) return 0.0;
    double u = 0.5 * cos(M_PI * r / rc) + 0.5;
    return u * u;
}
static double om_dfc(double r, double rc) {
    if (r >= rc) return 0.0;
    double u = 0.5 * cos(M_PI * r / rc) + 0.5;
    return 2.0 * u * (-0.5 * M_PI / rc * sin(M_PI * r / rc));
}

static double om_ipow(double x, int n) { double y = 1.0; for (int k = 0; k < n; ++k) y *= x; return y; }

/* Angular part A_lambda(d) and its gradient with respect to d (reading R4). */
static void om_angular(const om_lambda *q, double s, const double d[3], double *A, double (*dA)[3]) {
    double u[3] = { s * d[0], s * d[1], s * d[2] };
    for (int k = 0; k < q->n; ++k) {
        int lx = q->lx[k], ly = q->ly[k], lz = q->lz[k];
        double px = om_ipow(u[0], lx), py = om_ipow(u[1], ly), pz = om_ipow(u[2], lz);
        A[k] = px * py * pz;
        if (dA) {
            dA[k][0] = lx ? s * lx * om_ipow(u[0], lx - 1) * py * pz : 0.0;
            dA[k][1] = ly ? s * ly * px * om_ipow(u[1], ly - 1) * pz : 0.0;
            dA[k][2] = lz ? s * lz * px * py * om_ipow(u[2], lz - 1) : 0.0;
        }
    }
}

/* ------------------------------------------------------------ geometry -- */

static double om_wrap(double x, double L) {           /* reading R8 */
    double q = floor(x / L);
    double t = q * L;
    double w = x - t;
    if (w < 0.0) w = w + L;
    if (w >= L) w = w - L;
    return w;
}

static double om_dist2(const double d[3]) { return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0])); }

typedef struct {
    int64_t n_loc, n_ext, n_rows;
    int64_t *gid;     /* [n_ext] owner atom (global index) */
    int32_t *shift;   /* [n_ext][3] lattice shift of the copy */
    double *pos;      /* [n_ext][3] */
    int32_t *spec;    /* [n_ext] */
    int64_t *row;     /* [n_rows+1] */
    int64_t *col;     /* neighbour ext indices */
} om_domain;

static void om_domain_free(om_domain *D) {
    free(D->gid); free(D->shift); free(D->pos); free(D->spec); free(D->row); free(D->col);
    memset(D, 0, sizeof(*D));
}

typedef struct {
    int64_t n;
    double L[3];
    int per[3];
    int P[3];
    double *w;           /* [n][3] wrapped positions */
    int32_t *dom;        /* [n] flat subdomain index */
    double lo[3][64], hi[3][64];
} om_geom;

static int om_geom_init(om_geom *g, int64_t n, const double *pos, const double *cell, const int32_t *pbc,
                        const int32_t *decomp) {
    g->n = n;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            if (a != b && cell[3 * a + b] != 0.0) return OM_EINVAL;   /* orthorhombic only */
        g->L[a] = cell[4 * a];
        g->per[a] = pbc[a] ? 1 : 0;
        g->P[a] = decomp ? decomp[a] : 1;
        if (g->P[a] < 1 || g->P[a] > 64) return OM_EINVAL;
        if (!g->per[a] && g->P[a] != 1) return OM_EINVAL;
        if (g->per[a] && !(g->L[a] > 0.0)) return OM_EINVAL;
        if (g->per[a]) {
            double h = g->L[a] / g->P[a];
            for (int k = 0; k < g->P[a]; ++k) {
                g->lo[a][k] = k * h;
                g->hi[a][k] = (k == g->P[a] - 1) ? g->L[a] : (k + 1) * h;
            }
        } else {
            g->lo[a][0] = -INFINITY; g->hi[a][0] = INFINITY;
        }
    }
    g->w = malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    g->dom = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!g->w || !g->dom) return OM_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * i + a];
            if (!isfinite(x)) return OM_EINVAL;
            double w = g->per[a] ? om_wrap(x, g->L[a]) : x;
            g->w[3 * i + a] = w;
            c[a] = 0;
            for (int k = 0; k < g->P[a]; ++k)          /* the box that contains w */
                if (w >= g->lo[a][k] && w < g->hi[a][k]) c[a] = k;
        }
        g->dom[i] = (c[0] * g->P[1] + c[1]) * g->P[2] + c[2];
    }
    return OM_OK;
}

static void om_geom_free(om_geom *g) { free(g->w); free(g->dom); }

static int om_nmax(const om_geom *g, int a, double shell) {
    return g->per[a] ? (int)floor(shell / g->L[a]) + 1 : 0;
}

/* Locals and ghosts of subdomain p (reading R9; ghost shell `gshell` + 1e-6 around the box,
   gshell = rcut for the per-layer exchange), then the neighbour rows (cutoff rcut) of its
   locals (and of its ghosts when all_rows is set), each row sorted by ext index. */
static int om_domain_build(const om_geom *g, const int32_t *species, int p, double rcut, double gshell, int all_rows,
                           om_domain *D) {
    memset(D, 0, sizeof(*D));
    int pc[3] = { p / (g->P[1] * g->P[2]), (p / g->P[2]) % g->P[1], p % g->P[2] };
    double shell = gshell + 1e-6;
    int nm[3]; for (int a = 0; a < 3; ++a) nm[a] = om_nmax(g, a, shell);
    int64_t cap = 1024, n_ext = 0;
    D->gid = malloc(sizeof(int64_t) * cap); D->shift = malloc(sizeof(int32_t) * 3 * cap);
    D->pos = malloc(sizeof(double) * 3 * cap);
    if (!D->gid || !D->shift || !D->pos) return OM_ENOMEM;
#define OM_PUSH(o, s0, s1, s2, y0, y1, y2) do {                                              \
        if (n_ext == cap) {                                                                   \
            cap *= 2;                                                                         \
            D->gid = realloc(D->gid, sizeof(int64_t) * cap);                                  \
            D->shift = realloc(D->shift, sizeof(int32_t) * 3 * cap);                          \
            D->pos = realloc(D->pos, sizeof(double) * 3 * cap);                               \
            if (!D->gid || !D->shift || !D->pos) return OM_ENOMEM;                            \
        }                                                                                     \
        D->gid[n_ext] = (o); D->shift[3 * n_ext] = (s0); D->shift[3 * n_ext + 1] = (s1);      \
        D->shift[3 * n_ext + 2] = (s2); D->pos[3 * n_ext] = (y0); D->pos[3 * n_ext + 1] = (y1); \
        D->pos[3 * n_ext + 2] = (y2); ++n_ext;                                                \
    } while (0)
    for (int64_t o = 0; o < g->n; ++o)
        if (g->dom[o] == p) OM_PUSH(o, 0, 0, 0, g->w[3 * o], g->w[3 * o + 1], g->w[3 * o + 2]);
    D->n_loc = n_ext;
    for (int64_t o = 0; o < g->n; ++o)
        for (int s0 = -nm[0]; s0 <= nm[0]; ++s0)
            for (int s1 = -nm[1]; s1 <= nm[1]; ++s1)
                for (int s2 = -nm[2]; s2 <= nm[2]; ++s2) {
                    if (s0 == 0 && s1 == 0 && s2 == 0 && g->dom[o] == p) continue;
                    int s[3] = { s0, s1, s2 };
                    double y[3]; int in = 1;
                    for (int a = 0; a < 3; ++a) {
                        y[a] = g->per[a] ? g->w[3 * o + a] + (double)s[a] * g->L[a] : g->w[3 * o + a];
                        if (g->per[a] && !(y[a] >= g->lo[a][pc[a]] - shell && y[a] < g->hi[a][pc[a]] + shell))
                            in = 0;
                    }
                    if (in) OM_PUSH(o, s0, s1, s2, y[0], y[1], y[2]);
                }
#undef OM_PUSH
    D->n_ext = n_ext;
    D->spec = malloc(sizeof(int32_t) * (n_ext > 0 ? n_ext : 1));
    if (!D->spec) return OM_ENOMEM;
    for (int64_t e = 0; e < n_ext; ++e) D->spec[e] = species[D->gid[e]];

    /* plain cell binning over the bounding box of the ext copies, cells >= rcut */
    double mn[3], mx[3]; int nc[3]; double cs[3];
    for (int a = 0; a < 3; ++a) { mn[a] = INFINITY; mx[a] = -INFINITY; }
    for (int64_t e = 0; e < n_ext; ++e)
        for (int a = 0; a < 3; ++a) {
            if (D->pos[3 * e + a] < mn[a]) mn[a] = D->pos[3 * e + a];
            if (D->pos[3 * e + a] > mx[a]) mx[a] = D->pos[3 * e + a];
        }
    for (int a = 0; a < 3; ++a) {
        double ext = n_ext ? mx[a] - mn[a] : 0.0;
        nc[a] = (int)floor(ext / (rcut * 1.000001));
        if (nc[a] < 1) nc[a] = 1;
        if (nc[a] > 256) nc[a] = 256;
        cs[a] = nc[a] > 1 ? ext / nc[a] : 1.0;
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = malloc(sizeof(int64_t) * ncell), *next = malloc(sizeof(int64_t) * (n_ext + 1));
    int32_t *cell_of = malloc(sizeof(int32_t) * 3 * (n_ext + 1));
    if (!head || !next || !cell_of) return OM_ENOMEM;
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t e = n_ext - 1; e >= 0; --e) {
        int c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = nc[a] > 1 ? (int)((D->pos[3 * e + a] - mn[a]) / cs[a]) : 0;
            if (c[a] < 0) c[a] = 0;
            if (c[a] >= nc[a]) c[a] = nc[a] - 1;
            cell_of[3 * e + a] = c[a];
        }
        int64_t ci = ((int64_t)c[0] * nc[1] + c[1]) * nc[2] + c[2];
        next[e] = head[ci]; head[ci] = e;
    }
    D->n_rows = all_rows ? n_ext : D->n_loc;
    D->row = malloc(sizeof(int64_t) * (D->n_rows + 1));
    if (!D->row) return OM_ENOMEM;
    int64_t ccap = 1024, nn = 0;
    D->col = malloc(sizeof(int64_t) * ccap);
    int64_t *buf = malloc(sizeof(int64_t) * (n_ext + 1));
    if (!D->col || !buf) return OM_ENOMEM;
    double rc2 = rcut * rcut;
    D->row[0] = 0;
    for (int64_t i = 0; i < D->n_rows; ++i) {
        int64_t nb = 0;
        const int32_t *ci = cell_of + 3 * i;
        for (int c0 = ci[0] - 1; c0 <= ci[0] + 1; ++c0)
            for (int c1 = ci[1] - 1; c1 <= ci[1] + 1; ++c1)
                for (int c2 = ci[2] - 1; c2 <= ci[2] + 1; ++c2) {
                    if (c0 < 0 || c1 < 0 || c2 < 0 || c0 >= nc[0] || c1 >= nc[1] || c2 >= nc[2]) continue;
                    for (int64_t e = head[((int64_t)c0 * nc[1] + c1) * nc[2] + c2]; e >= 0; e = next[e]) {
                        if (e == i) continue;
                        double d[3] = { D->pos[3 * e] - D->pos[3 * i], D->pos[3 * e + 1] - D->pos[3 * i + 1],
                                        D->pos[3 * e + 2] - D->pos[3 * i + 2] };
                        if (om_dist2(d) < rc2) buf[nb++] = e;
                    }
                }
        /* insertion sort: rows in ext order */
        for (int64_t a = 1; a < nb; ++a) {
            int64_t v = buf[a], b = a - 1;
            while (b >= 0 && buf[b] > v) { buf[b + 1] = buf[b]; --b; }
            buf[b + 1] = v;
        }
        if (nn + nb > ccap) {
            while (nn + nb > ccap) ccap *= 2;
            D->col = realloc(D->col, sizeof(int64_t) * ccap);
            if (!D->col) return OM_ENOMEM;
        }
        memcpy(D->col + nn, buf, sizeof(int64_t) * nb);
        nn += nb;
        D->row[i + 1] = nn;
    }
    free(buf); free(head); free(next); free(cell_of);
    return OM_OK;
}

/* ------------------------------------------------------- neighbour export -- */

typedef struct { int64_t j; int32_t s[3]; } om_pair;

static int om_pair_cmp(const void *x, const void *y) {
    const om_pair *a = x, *b = y;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    for (int k = 0; k < 3; ++k) if (a->s[k] != b->s[k]) return a->s[k] < b->s[k] ? -1 : 1;
    return 0;
}

/* Neighbour list of every atom as (owner j, lattice shift) pairs, each row sorted by
   (j, shift), built through the subdomain decomposition `decomp` (NULL = whole).
   Two-call: with row == NULL returns the pair count; otherwise fills row[n+1],
   j[count], shift[count][3] and returns the count.  Negative = error. */
int64_t oracle_neighbors(int64_t n, const double *pos, const double *cell, const int32_t *pbc, double rcut,
                         const int32_t *decomp, int64_t *row, int64_t *jout, int32_t *sout) {
    if (n < 0 || !pos || !cell || !pbc || !(rcut > 0.0)) return OM_EINVAL;
    om_geom g; memset(&g, 0, sizeof g);
    int rc = om_geom_init(&g, n, pos, cell, pbc, decomp);
    if (rc) { om_geom_free(&g); return rc; }
    int np = g.P[0] * g.P[1] * g.P[2];
    int32_t *zero_spec = calloc(n > 0 ? n : 1, sizeof(int32_t));
    int64_t *cnt = calloc(n + 1, sizeof(int64_t));
    om_pair **rows = calloc(n > 0 ? n : 1, sizeof(om_pair *));
    for (int p = 0; p < np; ++p) {
        om_domain D;
        rc = om_domain_build(&g, zero_spec, p, rcut, rcut, 0, &D);
        if (rc) { om_domain_free(&D); break; }
        for (int64_t i = 0; i < D.n_loc; ++i) {
            int64_t gi = D.gid[i], nb = D.row[i + 1] - D.row[i];
            cnt[gi] = nb;
            rows[gi] = malloc(sizeof(om_pair) * (nb > 0 ? nb : 1));
            for (int64_t k = 0; k < nb; ++k) {
                int64_t e = D.col[D.row[i] + k];
                rows[gi][k].j = D.gid[e];
                for (int a = 0; a < 3; ++a) rows[gi][k].s[a] = D.shift[3 * e + a];
            }
            qsort(rows[gi], nb, sizeof(om_pair), om_pair_cmp);
        }
        om_domain_free(&D);
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += cnt[i];
    if (rc == OM_OK && row) {
        row[0] = 0;
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t k = 0; k < cnt[i]; ++k) {
                jout[row[i] + k] = rows[i][k].j;
                for (int a = 0; a < 3; ++a) sout[3 * (row[i] + k) + a] = rows[i][k].s[a];
            }
            row[i + 1] = row[i] + cnt[i];
        }
    }
    for (int64_t i = 0; i < n; ++i) free(rows[i]);
    free(rows); free(cnt); free(zero_spec); om_geom_free(&g);
    return rc ? rc : total;
}

/* ------------------------------------------------------------ evaluation -- */

typedef struct {
    const om_model *m;
    om_lambda q;
    int K, F, NL;
} om_ctx;

/* Orbital sums of row atom a of domain D (Eq. (1) inner sum, readings R2-R4):
   S[lambda][m] = sum_j c_j[m] A_lambda(d_aj) R_m(r_aj) f_c(r_aj). */
static void om_edge_sum(const om_ctx *C, const om_domain *D, int64_t a, const double *c_ext, double *S) {
    const om_model *m = C->m;
    int K = C->K, NL = C->NL;
    double A[64];
    memset(S, 0, sizeof(double) * NL * K);
    for (int64_t k = D->row[a]; k < D->row[a + 1]; ++k) {
        int64_t e = D->col[k];
        double d[3] = { D->pos[3 * e] - D->pos[3 * a], D->pos[3 * e + 1] - D->pos[3 * a + 1],
                        D->pos[3 * e + 2] - D->pos[3 * a + 2] };
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r >= m->r_c) continue;
        double fc = om_fc(r, m->r_c);
        om_angular(&C->q, m->ang_scale, d, A, NULL);
        for (int mm = 0; mm < K; ++mm) {
            double x = r - m->centres[mm];
            double w = c_ext[e * K + mm] * exp(-m->alphas[mm] * x * x) * fc;
            for (int l = 0; l < NL; ++l) S[l * K + mm] += w * A[l];
        }
    }
}

/* Adjoint of om_edge_sum for one edge a->e given Sbar_a: accumulates the force on a
   (+g) and on e (-g), the message adjoint cbar_e, and the virial -d (x) g (reading R6). */
static void om_edge_adjoint(const om_ctx *C, const double *da, const double *de, const double *Sbar,
                            const double *ce, double *Fa, double *Fe, double *cbar_e, double *W) {
    const om_model *m = C->m;
    int K = C->K, NL = C->NL;
    double d[3] = { de[0] - da[0], de[1] - da[1], de[2] - da[2] };
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r >= m->r_c) return;
    double fc = om_fc(r, m->r_c), dfc = om_dfc(r, m->r_c);
    double A[64], dA[64][3];
    om_angular(&C->q, m->ang_scale, d, A, dA);
    double g[3] = { 0, 0, 0 };
    for (int mm = 0; mm < K; ++mm) {
        double x = r - m->centres[mm];
        double R = exp(-m->alphas[mm] * x * x);
        double dR = -2.0 * m->alphas[mm] * x * R;
        double cb = 0.0;
        for (int l = 0; l < NL; ++l) {
            double s = Sbar[l * K + mm];
            double a = s * ce[mm];
            double radial = dR * fc + R * dfc;   /* d(R f_c)/dr */
            for (int k = 0; k < 3; ++k) g[k] += a * (dA[l][k] * R * fc + A[l] * radial * d[k] / r);
            cb += s * A[l] * R * fc;
        }
        if (cbar_e) cbar_e[mm] += cb;
    }
    for (int k = 0; k < 3; ++k) { Fa[k] += g[k]; Fe[k] -= g[k]; }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) W[3 * a + b] -= d[a] * g[b];
}

/* Energy, forces and virial (see the readings at the top).
 *   decomp  subdomains per axis (NULL = 1,1,1 = whole system with periodic images as ghosts)
 *   naive   negative control: ghosts' messages are computed inside each subdomain from its
 *           incomplete neighbourhood instead of being copied from their owners (Sec. 2.2,
 *           the failure the paper describes); energy only.
 *   outputs energy (required), atom_energy[n], forces[n][3], virial[9] (row-major W_ab),
 *           S_out[T][n][NL][K] and c_out[T][n][K] (debug, per layer, global atom order);
 *           each may be NULL. */
int oracle_eval(const om_model *m, int64_t n, const double *pos, const int32_t *species, const double *cell,
                const int32_t *pbc, double skin, int32_t T, const int32_t *decomp, int32_t naive,
                int32_t n_threads, double *energy, double *atom_energy, double *forces, double *virial,
                double *S_out, double *c_out) {
    if (!m || !pos || !species || !cell || !pbc || !energy || n <= 0) return OM_EINVAL;
    if (T < 1 || T > m->T_max || m->K < 1 || m->K > 64 || m->L < 0 || m->L > 4 || !(m->r_c > 0.0) ||
        skin < 0.0 || m->hidden > 1024 || m->n_hidden > 7 || m->n_hidden < 0)
        return OM_EINVAL;
    for (int64_t i = 0; i < n; ++i) if (species[i] < 0 || species[i] >= m->n_species) return OM_EINVAL;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    if (m->form != OM_FORM_REANN && m->form != OM_FORM_DIAG && !(m->form == OM_FORM_RADIAL && m->L == 0))
        return OM_EINVAL;
    const int radial = m->form == OM_FORM_RADIAL;
    om_ctx C; C.m = m; om_lambda_init(m->L, &C.q);
    C.K = m->K; C.F = om_model_nfeat(m); C.NL = C.q.n;
    const int K = C.K, F = C.F, NL = C.NL, H = m->hidden, nh = m->n_hidden;
    if (F > 1024) return OM_EINVAL;

    om_geom g; memset(&g, 0, sizeof g);
    int rc = om_geom_init(&g, n, pos, cell, pbc, decomp);
    if (rc) { om_geom_free(&g); return rc; }
    int np = g.P[0] * g.P[1] * g.P[2];
    double rcut = m->r_c + skin;
    om_domain *D = calloc(np, sizeof(om_domain));
    for (int p = 0; p < np && rc == OM_OK; ++p) rc = om_domain_build(&g, species, p, rcut, rcut, naive, &D[p]);
    if (rc) goto done;

    /* per domain, per layer: messages of every ext atom; orbital sums of locals */
    double ***c = calloc(np, sizeof(double **)), ***S = calloc(np, sizeof(double **));
    double *cglob = calloc((size_t)n * K, sizeof(double));
    double *Eat = calloc(n, sizeof(double));
    for (int p = 0; p < np; ++p) {
        c[p] = calloc(T, sizeof(double *)); S[p] = calloc(T, sizeof(double *));
        for (int t = 0; t < T; ++t) {
            c[p][t] = calloc((size_t)D[p].n_ext * K + 1, sizeof(double));
            S[p][t] = calloc((size_t)D[p].n_loc * NL * K + 1, sizeof(double));
        }
        for (int64_t e = 0; e < D[p].n_ext; ++e)             /* c^0: per element (R2) */
            for (int k = 0; k < K; ++k) c[p][0][e * K + k] = m->c0[D[p].spec[e] * K + k];
    }

    for (int t = 0; t < T; ++t) {
        for (int p = 0; p < np; ++p) {
            om_domain *Dp = &D[p];
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t i = 0; i < Dp->n_loc; ++i) om_edge_sum(&C, Dp, i, c[p][t], S[p][t] + i * NL * K);
        }
        if (t == T - 1) break;
        /* message update of the locals, Eq. (2) */
        for (int p = 0; p < np; ++p) {
            om_domain *Dp = &D[p];
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t i = 0; i < Dp->n_loc; ++i) {
                double rho[1024];
                om_features(m, &C.q, S[p][t] + i * NL * K, rho);
                double *ci = cglob + Dp->gid[i] * K;
                om_mlp_forward(om_msg_params(m, t, Dp->spec[i]), F, H, nh, K, rho, ci);
                if (radial)   /* residual update (reading R14) */
                    for (int k = 0; k < K; ++k) ci[k] += c[p][t][i * K + k];
            }
        }
        for (int p = 0; p < np; ++p) {
            om_domain *Dp = &D[p];
            /* locals keep their own value; ghosts receive their owner's (the per-layer exchange) */
            for (int64_t e = 0; e < Dp->n_ext; ++e)
                memcpy(c[p][t + 1] + e * K, cglob + Dp->gid[e] * K, sizeof(double) * K);
            if (naive) {
                /* negative control: recompute ghosts' messages from the subdomain's own data */
#pragma omp parallel for schedule(dynamic, 64)
                for (int64_t e = Dp->n_loc; e < Dp->n_ext; ++e) {
                    double Sg[64 * 35], rho[1024];
                    om_edge_sum(&C, Dp, e, c[p][t], Sg);
                    om_features(m, &C.q, Sg, rho);
                    om_mlp_forward(om_msg_params(m, t, Dp->spec[e]), F, H, nh, K, rho, c[p][t + 1] + e * K);
                    if (radial)
                        for (int k = 0; k < K; ++k) c[p][t + 1][e * K + k] += c[p][t][e * K + k];
                }
            }
        }
    }
    /* atomic energies (R5) */
    for (int p = 0; p < np; ++p) {
        om_domain *Dp = &D[p];
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < Dp->n_loc; ++i) {
            double rho[1024], y;
            om_features(m, &C.q, S[p][T - 1] + i * NL * K, rho);
            om_mlp_forward(om_en_params(m, Dp->spec[i]), F, H, nh, 1, rho, &y);
            Eat[Dp->gid[i]] = m->energy_scale * y;
        }
    }
    double Etot = 0.0;
    for (int64_t i = 0; i < n; ++i) Etot += Eat[i];
    *energy = Etot;
    if (atom_energy) memcpy(atom_energy, Eat, sizeof(double) * n);
    if (S_out || c_out)
        for (int p = 0; p < np; ++p)
            for (int t = 0; t < T; ++t)
                for (int64_t i = 0; i < D[p].n_loc; ++i) {
                    int64_t gi = D[p].gid[i];
                    if (S_out) memcpy(S_out + ((size_t)t * n + gi) * NL * K, S[p][t] + i * NL * K, sizeof(double) * NL * K);
                    if (c_out) memcpy(c_out + ((size_t)t * n + gi) * K, c[p][t] + i * K, sizeof(double) * K);
                }

    if ((forces || virial) && !naive) {
        /* backward, Eqs. (3)-(5) */
        double **Sbar = calloc(np, sizeof(double *)), **Fext = calloc(np, sizeof(double *));
        double **cbar = calloc(np, sizeof(double *));
        double *cbglob = calloc((size_t)n * K, sizeof(double));
        /* radial form: dE/dc^{t+1} of every atom, carried into dE/dc^t by the residual */
        double *cbnext = calloc((size_t)n * K, sizeof(double));
        double Wtot[9] = { 0 };
        for (int p = 0; p < np; ++p) {
            Sbar[p] = calloc((size_t)D[p].n_loc * NL * K + 1, sizeof(double));
            Fext[p] = calloc((size_t)D[p].n_ext * 3 + 1, sizeof(double));
            cbar[p] = calloc((size_t)D[p].n_ext * K + 1, sizeof(double));
            om_domain *Dp = &D[p];
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t i = 0; i < Dp->n_loc; ++i) {
                double rho[1024], rhobar[1024], ybar = m->energy_scale;
                om_features(m, &C.q, S[p][T - 1] + i * NL * K, rho);
                om_mlp_vjp(om_en_params(m, Dp->spec[i]), F, H, nh, 1, rho, &ybar, rhobar);
                om_features_vjp(m, &C.q, S[p][T - 1] + i * NL * K, rhobar, Sbar[p] + i * NL * K);
            }
        }
        for (int t = T - 1; t >= 0; --t) {
            for (int p = 0; p < np; ++p) {
                om_domain *Dp = &D[p];
                memset(cbar[p], 0, sizeof(double) * Dp->n_ext * K);
                int nthr = 1;
#ifdef _OPENMP
                nthr = omp_get_max_threads();
#endif
                double *privF = calloc((size_t)nthr * Dp->n_ext * 3 + 1, sizeof(double));
                double *privC = calloc((size_t)nthr * Dp->n_ext * K + 1, sizeof(double));
                double *privW = calloc((size_t)nthr * 9, sizeof(double));
#pragma omp parallel
                {
                    int tid = 0;
#ifdef _OPENMP
                    tid = omp_get_thread_num();
#endif
                    double *pF = privF + (size_t)tid * Dp->n_ext * 3, *pC = privC + (size_t)tid * Dp->n_ext * K;
#pragma omp for schedule(dynamic, 64)
                    for (int64_t i = 0; i < Dp->n_loc; ++i)
                        for (int64_t k = Dp->row[i]; k < Dp->row[i + 1]; ++k) {
                            int64_t e = Dp->col[k];
                            om_edge_adjoint(&C, Dp->pos + 3 * i, Dp->pos + 3 * e, Sbar[p] + i * NL * K,
                                            c[p][t] + e * K, pF + 3 * i, pF + 3 * e, t > 0 ? pC + e * K : NULL,
                                            privW + 9 * tid);
                        }
                }
                for (int th = 0; th < nthr; ++th) {
                    for (int64_t x = 0; x < Dp->n_ext * 3; ++x) Fext[p][x] += privF[(size_t)th * Dp->n_ext * 3 + x];
                    if (t > 0)
                        for (int64_t x = 0; x < Dp->n_ext * K; ++x) cbar[p][x] += privC[(size_t)th * Dp->n_ext * K + x];
                    for (int x = 0; x < 9; ++x) Wtot[x] += privW[9 * th + x];
                }
                free(privF); free(privC); free(privW);
            }
            if (t == 0) break;                       /* dc^0/dr = 0 */
            /* reverse exchange: ghost message adjoints summed onto their owners */
            memset(cbglob, 0, sizeof(double) * n * K);
            for (int p = 0; p < np; ++p)
                for (int64_t e = 0; e < D[p].n_ext; ++e)
                    for (int k = 0; k < K; ++k) cbglob[D[p].gid[e] * K + k] += cbar[p][e * K + k];
            if (radial) {
                /* c^t also reaches the energy through c^{t+1} = c^t + M(x^t) when t < T-1 */
                if (t < T - 1)
                    for (int64_t x = 0; x < n * K; ++x) cbglob[x] += cbnext[x];
                memcpy(cbnext, cbglob, sizeof(double) * n * K);
            }
            for (int p = 0; p < np; ++p) {
                om_domain *Dp = &D[p];
#pragma omp parallel for schedule(dynamic, 64)
                for (int64_t i = 0; i < Dp->n_loc; ++i) {
                    double rho[1024], rhobar[1024];
                    om_features(m, &C.q, S[p][t - 1] + i * NL * K, rho);
                    om_mlp_vjp(om_msg_params(m, t - 1, Dp->spec[i]), F, H, nh, K, rho, cbglob + Dp->gid[i] * K, rhobar);
                    om_features_vjp(m, &C.q, S[p][t - 1] + i * NL * K, rhobar, Sbar[p] + i * NL * K);
                }
            }
        }
        if (forces) {
            memset(forces, 0, sizeof(double) * n * 3);
            for (int p = 0; p < np; ++p)           /* ghost forces summed onto their owners */
                for (int64_t e = 0; e < D[p].n_ext; ++e)
                    for (int k = 0; k < 3; ++k) forces[D[p].gid[e] * 3 + k] += Fext[p][e * 3 + k];
        }
        if (virial) memcpy(virial, Wtot, sizeof(Wtot));
        for (int p = 0; p < np; ++p) { free(Sbar[p]); free(Fext[p]); free(cbar[p]); }
        free(Sbar); free(Fext); free(cbar); free(cbglob); free(cbnext);
    }

    for (int p = 0; p < np; ++p) {
        for (int t = 0; t < T; ++t) { free(c[p][t]); free(S[p][t]); }
        free(c[p]); free(S[p]);
    }
    free(c); free(S); free(cglob); free(Eat);
done:
    for (int p = 0; p < np; ++p) om_domain_free(&D[p]);
    free(D);
    om_geom_free(&g);
    return rc;
}

/* ------------------------------------------------- extended-halo scheme -- */

/* Halo level of ext copy e of subdomain p: 0 for the locals, else the smallest k >= 1 such
   that the copy lies within k rcut + 1e-6 of the box on every split or periodic axis (the shell
   test of reading R9 with k rcut for r_c + skin).  A neighbour (distance < rcut) of a copy of
   level k has level <= k + 1. */
static int om_halo_level(const om_geom *g, const om_domain *D, int p, int64_t e, double rcut) {
    if (e < D->n_loc) return 0;
    int pc[3] = { p / (g->P[1] * g->P[2]), (p / g->P[2]) % g->P[1], p % g->P[2] };
    for (int k = 1;; ++k) {
        double s = k * rcut + 1e-6;
        int in = 1;
        for (int a = 0; a < 3; ++a) {
            double y = D->pos[3 * e + a];
            if (g->per[a] && !(y >= g->lo[a][pc[a]] - s && y < g->hi[a][pc[a]] + s)) in = 0;
        }
        if (in) return k;
    }
}

/* Energy, forces and virial by the extended-halo scheme: the alternative to the per-layer
 * exchange that the paper argues against (Sec. 2.2, Fig. 2(a): the receptive field of T layers
 * reaches T r_c).  Each subdomain takes every copy within T (r_c + skin) of its box and runs the
 * T layers with no exchange between them: layer t evaluates every copy of halo level at most
 * T - 1 - t (those are the atoms whose layer-t output reaches a local's energy), reading its
 * neighbours' layer-t messages from the same subdomain.  E_p sums the locals' atomic energies
 * and E = sum_p E_p; the reverse sweep runs inside each subdomain over the same copies, the
 * message adjoints staying there, and the copies' forces are summed onto their owners once at
 * the end.  It must give the whole-system E, F and W; the cost is the redundant evaluation of
 * the halo copies.
 *   work (optional) [T][2]: rows evaluated and in-cutoff edges summed, per layer, over all
 *   subdomains (the per-layer exchange evaluates n rows and the locals' edges per layer). */
int oracle_eval_halo(const om_model *m, int64_t n, const double *pos, const int32_t *species, const double *cell,
                     const int32_t *pbc, double skin, int32_t T, const int32_t *decomp, int32_t n_threads,
                     double *energy, double *atom_energy, double *forces, double *virial, int64_t *work) {
    if (!m || !pos || !species || !cell || !pbc || !energy || n <= 0) return OM_EINVAL;
    if (T < 1 || T > m->T_max || m->K < 1 || m->K > 64 || m->L < 0 || m->L > 4 || !(m->r_c > 0.0) ||
        skin < 0.0 || m->hidden > 1024 || m->n_hidden > 7 || m->n_hidden < 0)
        return OM_EINVAL;
    for (int64_t i = 0; i < n; ++i) if (species[i] < 0 || species[i] >= m->n_species) return OM_EINVAL;
    if (m->form != OM_FORM_REANN) return OM_EINVAL;   /* the ablation is kept to the paper's form */
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    om_ctx C; C.m = m; om_lambda_init(m->L, &C.q);
    C.K = m->K; C.F = om_nfeat(m->L, m->K); C.NL = C.q.n;
    const int K = C.K, F = C.F, NL = C.NL, H = m->hidden, nh = m->n_hidden;
    if (F > 1024) return OM_EINVAL;
    om_geom g; memset(&g, 0, sizeof g);
    int rc = om_geom_init(&g, n, pos, cell, pbc, decomp);
    if (rc) { om_geom_free(&g); return rc; }
    int np = g.P[0] * g.P[1] * g.P[2];
    double rcut = m->r_c + skin;
    double *Eat = calloc(n, sizeof(double));
    double Wtot[9] = { 0 };
    if (forces) memset(forces, 0, sizeof(double) * n * 3);
    if (work) memset(work, 0, sizeof(int64_t) * 2 * T);
    for (int p = 0; p < np && rc == OM_OK; ++p) {
        om_domain D;
        rc = om_domain_build(&g, species, p, rcut, T * rcut, 1, &D);
        if (rc) { om_domain_free(&D); break; }
        const int64_t ne = D.n_ext;
        int *lev = malloc(sizeof(int) * (ne + 1));
        for (int64_t e = 0; e < ne; ++e) lev[e] = om_halo_level(&g, &D, p, e, rcut);
        double **c = calloc(T, sizeof(double *)), **S = calloc(T, sizeof(double *));
        for (int t = 0; t < T; ++t) {
            c[t] = calloc((size_t)ne * K + 1, sizeof(double));
            S[t] = calloc((size_t)ne * NL * K + 1, sizeof(double));
        }
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < K; ++k) c[0][e * K + k] = m->c0[D.spec[e] * K + k];
        for (int t = 0; t < T; ++t) {
            const int top = T - 1 - t;   /* rows of level <= top are evaluated at layer t */
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t e = 0; e < ne; ++e) {
                if (lev[e] > top) continue;
                om_edge_sum(&C, &D, e, c[t], S[t] + e * NL * K);
                if (t < T - 1) {
                    double rho[1024];
                    om_features(m, &C.q, S[t] + e * NL * K, rho);
                    om_mlp_forward(om_msg_params(m, t, D.spec[e]), F, H, nh, K, rho, c[t + 1] + e * K);
                }
            }
            if (work)
                for (int64_t e = 0; e < ne; ++e) {
                    if (lev[e] > top) continue;
                    work[2 * t] += 1;
                    for (int64_t k = D.row[e]; k < D.row[e + 1]; ++k) {
                        int64_t j = D.col[k];
                        double d[3] = { D.pos[3 * j] - D.pos[3 * e], D.pos[3 * j + 1] - D.pos[3 * e + 1],
                                        D.pos[3 * j + 2] - D.pos[3 * e + 2] };
                        if (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < m->r_c) work[2 * t + 1] += 1;
                    }
                }
        }
        for (int64_t i = 0; i < D.n_loc; ++i) {
            double rho[1024], y;
            om_features(m, &C.q, S[T - 1] + i * NL * K, rho);
            om_mlp_forward(om_en_params(m, D.spec[i]), F, H, nh, 1, rho, &y);
            Eat[D.gid[i]] = m->energy_scale * y;
        }
        if (forces || virial) {
            double *Sbar = calloc((size_t)ne * NL * K + 1, sizeof(double));
            double *Fext = calloc((size_t)ne * 3 + 1, sizeof(double));
            double *cbar = calloc((size_t)ne * K + 1, sizeof(double));
            for (int64_t i = 0; i < D.n_loc; ++i) {
                double rho[1024], rhobar[1024], ybar = m->energy_scale;
                om_features(m, &C.q, S[T - 1] + i * NL * K, rho);
                om_mlp_vjp(om_en_params(m, D.spec[i]), F, H, nh, 1, rho, &ybar, rhobar);
                om_features_vjp(m, &C.q, S[T - 1] + i * NL * K, rhobar, Sbar + i * NL * K);
            }
            for (int t = T - 1; t >= 0; --t) {
                const int top = T - 1 - t;
                memset(cbar, 0, sizeof(double) * ne * K);
                /* serial over rows: every edge adds to both ends, in row order */
                for (int64_t e = 0; e < ne; ++e) {
                    if (lev[e] > top) continue;
                    for (int64_t k = D.row[e]; k < D.row[e + 1]; ++k) {
                        int64_t j = D.col[k];
                        om_edge_adjoint(&C, D.pos + 3 * e, D.pos + 3 * j, Sbar + e * NL * K, c[t] + j * K, Fext + 3 * e,
                                        Fext + 3 * j, t > 0 ? cbar + j * K : NULL, Wtot);
                    }
                }
                if (t == 0) break;                   /* dc^0/dr = 0 */
                /* message adjoints stay in the subdomain: through layer t-1's message NN of
                   every row evaluated there */
                memset(Sbar, 0, sizeof(double) * ne * NL * K);
#pragma omp parallel for schedule(dynamic, 64)
                for (int64_t e = 0; e < ne; ++e) {
                    if (lev[e] > T - t) continue;
                    double rho[1024], rhobar[1024];
                    om_features(m, &C.q, S[t - 1] + e * NL * K, rho);
                    om_mlp_vjp(om_msg_params(m, t - 1, D.spec[e]), F, H, nh, K, rho, cbar + e * K, rhobar);
                    om_features_vjp(m, &C.q, S[t - 1] + e * NL * K, rhobar, Sbar + e * NL * K);
                }
            }
            if (forces)                                /* copies' forces summed onto their owners */
                for (int64_t e = 0; e < ne; ++e)
                    for (int k = 0; k < 3; ++k) forces[D.gid[e] * 3 + k] += Fext[e * 3 + k];
            free(Sbar); free(Fext); free(cbar);
        }
        for (int t = 0; t < T; ++t) { free(c[t]); free(S[t]); }
        free(c); free(S); free(lev);
        om_domain_free(&D);
    }
    if (rc == OM_OK) {
        double Etot = 0.0;
        for (int64_t i = 0; i < n; ++i) Etot += Eat[i];
        *energy = Etot;
        if (atom_energy) memcpy(atom_energy, Eat, sizeof(double) * n);
        if (virial) memcpy(virial, Wtot, sizeof(Wtot));
    }
    free(Eat);
    om_geom_free(&g);
    return rc;
}

/* Sizes the caller needs for the debug outputs. */
int oracle_dims(int32_t L, int32_t K, int32_t *n_lambda, int32_t *n_feat) {
    if (n_lambda) *n_lambda = om_nlambda(L);
    if (n_feat) *n_feat = om_nfeat(L, K);
    return 0;
}
