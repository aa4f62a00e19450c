/*
 * FP64 CPU oracle for the SPH density and force pair interactions.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header or table with the GPU library and must never be called from it.
 *
 * What it computes is the plain definition of the two stages of Section II
 * (Algorithms): for every particle i, the density sums over all j within
 * h_i, and the force sums over all j within max(h_i, h_j), on a periodic
 * box with the minimum-image convention (Section II-B: pairs across periodic
 * boundaries).  The paper does not print the SPH formulas; the readings used
 * here (cubic-spline kernel with support h, grad-h density/force in the form
 * of the paper's comparison code, Monaghan signal-velocity viscosity with
 * alpha from Section III-B) are listed with their reasons in the design notes
 * of the repository.  Everything is IEEE FP64, round-to-nearest, no
 * fast-math.
 *
 * Neighbour search is exact and obviously so:
 *   * brute force: every j is tested;
 *   * grid: particles are bucketed into classes by their own h (class c holds
 *     box/2^(c+1) < h <= box/2^c) and, within a class, sorted by a 21-bit
 *     per-axis Morton key.  A query of radius R against class c uses the
 *     octree level whose cells are at least R wide and scans the 27 cells
 *     around the target (all particles of the class when that level has
 *     fewer than 3 cells per side).  Any j within R of i under the minimum
 *     image then lies in one of those 27 cells.
 * Both modes visit neighbours in a fixed order, so the results do not depend
 * on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_E_ARG (-1)
#define ORA_E_NOCONV (-5)
#define ORA_E_MEM (-8)

static const double ORA_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------------
 * Cubic spline (M4) with support radius h, normalised to unit volume
 * integral: W(r,h) = 8/(pi h^3) f(r/h).
 * ------------------------------------------------------------------------- */
double ora_kernel_f(double q) {
    if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) { double t = 1.0 - q; return 2.0 * t * t * t; }
    return 0.0;
}

double ora_kernel_df(double q) {          /* f'(q) */
    if (q < 0.5) return -12.0 * q + 18.0 * q * q;
    if (q < 1.0) { double t = 1.0 - q; return -6.0 * t * t; }
    return 0.0;
}

double ora_W(double r, double h) { return 8.0 / (ORA_PI * h * h * h) * ora_kernel_f(r / h); }

/* dW/dh at fixed r: -8/(pi h^4) (3 f(q) + q f'(q)) */
double ora_dWdh(double r, double h) {
    double q = r / h;
    return -8.0 / (ORA_PI * h * h * h * h) * (3.0 * ora_kernel_f(q) + q * ora_kernel_df(q));
}

/* Scalar k with grad_i W(|x_ij|, h) = k * x_ij, i.e. k = W'(r)/r. */
double ora_gradW_factor(double r, double h) {
    if (r <= 0.0 || r >= h) return 0.0;
    double q = r / h;
    return 8.0 / (ORA_PI * h * h * h * h) * ora_kernel_df(q) / r;
}

/* splitmix64 output function applied to (id + golden gamma): the per-id
 * hash summed mod 2^64 over a particle's neighbour set. */
uint64_t ora_mix(uint64_t id) {
    uint64_t z = id + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ---------------------------------------------------------------------------
 * Particle set and the exact neighbour search.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    double box;
} ora_pos;

static inline double min_image(double d, double box) { return d - box * nearbyint(d / box); }

#define KBITS 21
#define KRES (1 << KBITS)

static inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFF;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
static inline uint64_t morton3(uint64_t a, uint64_t b, uint64_t c) {
    return (spread3(a) << 2) | (spread3(b) << 1) | spread3(c);
}

static inline int64_t cell_coord(double x, double box, int64_t G) {
    double w = x - box * floor(x / box);       /* wrap into [0, box) */
    int64_t k = (int64_t)floor(w / box * (double)G);
    if (k < 0) k = 0;
    if (k >= G) k = G - 1;
    return k;
}

typedef struct { uint64_t key; int64_t idx; } kv;

static int kv_cmp(const void* a, const void* b) {
    const kv *p = (const kv*)a, *q = (const kv*)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

typedef struct {
    int ncls;
    int64_t start[KBITS + 2];   /* class c occupies [start[c], start[c+1]) */
    double hmax[KBITS + 1];     /* largest h in class c (0 if empty) */
    kv* e;
} ora_grid;

static int class_of(double h, double box) {
    /* class c: box/2^(c+1) < h <= box/2^c ; very small h go to the last */
    int c = 0;
    double edge = box;
    while (c < KBITS && h <= 0.5 * edge) { edge *= 0.5; ++c; }
    return c;
}

/* by_h = 0: one class holding every particle (density needs no h_j). */
static int grid_build(ora_grid* g, const ora_pos* p, const double* h, int by_h) {
    int64_t n = p->n;
    g->ncls = by_h ? KBITS + 1 : 1;
    g->e = (kv*)malloc(sizeof(kv) * (size_t)(n > 0 ? n : 1));
    if (!g->e) return ORA_E_MEM;
    int* cls = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!cls) { free(g->e); return ORA_E_MEM; }
    int64_t cnt[KBITS + 2];
    memset(cnt, 0, sizeof(cnt));
    for (int c = 0; c <= KBITS; ++c) g->hmax[c] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int c = by_h ? class_of(h[i], p->box) : 0;
        cls[i] = c;
        cnt[c]++;
        if (by_h && h[i] > g->hmax[c]) g->hmax[c] = h[i];
    }
    g->start[0] = 0;
    for (int c = 0; c < g->ncls; ++c) g->start[c + 1] = g->start[c] + cnt[c];
    int64_t fill[KBITS + 2];
    memcpy(fill, g->start, sizeof(fill));
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix = cell_coord(p->x[i], p->box, KRES);
        int64_t iy = cell_coord(p->y[i], p->box, KRES);
        int64_t iz = cell_coord(p->z[i], p->box, KRES);
        kv v = { morton3((uint64_t)ix, (uint64_t)iy, (uint64_t)iz), i };
        g->e[fill[cls[i]]++] = v;
    }
    free(cls);
    for (int c = 0; c < g->ncls; ++c)
        qsort(g->e + g->start[c], (size_t)(g->start[c + 1] - g->start[c]), sizeof(kv), kv_cmp);
    return ORA_OK;
}

static void grid_free(ora_grid* g) { free(g->e); g->e = NULL; }

static int64_t lower_key(const kv* e, int64_t lo, int64_t hi, uint64_t key) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (e[mid].key < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Visit every particle of class c that may lie within R of point (xi,yi,zi):
 * the visitor gets candidate indices; it applies the exact distance test.
 * Order of visits is deterministic. */
typedef void (*visit_fn)(int64_t j, void* ctx);

static void grid_query(const ora_grid* g, const ora_pos* p, int c, double xi, double yi, double zi,
                       double R, visit_fn fn, void* ctx) {
    int64_t s = g->start[c], t = g->start[c + 1];
    if (s == t) return;
    int lvl = 0;
    double edge = p->box;
    while (lvl < KBITS && 0.5 * edge >= R) { edge *= 0.5; ++lvl; }
    int64_t G = (int64_t)1 << lvl;
    if (G < 3) {
        for (int64_t k = s; k < t; ++k) fn(g->e[k].idx, ctx);
        return;
    }
    int64_t cx = cell_coord(xi, p->box, G), cy = cell_coord(yi, p->box, G), cz = cell_coord(zi, p->box, G);
    int shift = 3 * (KBITS - lvl);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                uint64_t ax = (uint64_t)((cx + dx + G) % G);
                uint64_t ay = (uint64_t)((cy + dy + G) % G);
                uint64_t az = (uint64_t)((cz + dz + G) % G);
                uint64_t code = morton3(ax, ay, az);   /* level-lvl coords, bits < lvl */
                uint64_t k0 = code << shift, k1 = (code + 1) << shift;
                int64_t a = lower_key(g->e, s, t, k0);
                int64_t b = lower_key(g->e, a, t, k1);
                for (int64_t k = a; k < b; ++k) fn(g->e[k].idx, ctx);
            }
}

/* ---------------------------------------------------------------------------
 * Density stage (Section II, item 1): sums over j != i with r_ij < h_i,
 * plus the self term.
 * ------------------------------------------------------------------------- */
typedef struct {
    const ora_pos* p;
    const double* m;
    int64_t i;
    double hi;
    double sf, sg, sw, sqdf;   /* sum m f, sum m g, sum f, sum q f' */
    int64_t nn;
    uint64_t hash;
} dens_ctx;

static void dens_visit(int64_t j, void* vctx) {
    dens_ctx* c = (dens_ctx*)vctx;
    if (j == c->i) return;
    const ora_pos* p = c->p;
    double dx = min_image(p->x[c->i] - p->x[j], p->box);
    double dy = min_image(p->y[c->i] - p->y[j], p->box);
    double dz = min_image(p->z[c->i] - p->z[j], p->box);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(r < c->hi)) return;
    double q = r / c->hi;
    double f = ora_kernel_f(q), df = ora_kernel_df(q);
    c->sf += c->m[j] * f;
    c->sg += c->m[j] * (3.0 * f + q * df);
    c->sw += f;
    c->sqdf += q * df;
    c->nn += 1;
    c->hash += ora_mix((uint64_t)j);
}

static void density_one(const ora_pos* p, const ora_grid* g, const double* m, int64_t i, double hi,
                        double* rho, double* drho, double* nw, double* dnw, int64_t* nn, uint64_t* hash) {
    dens_ctx c = { p, m, i, hi, 0, 0, 0, 0, 0, 0 };
    if (g) {
        grid_query(g, p, 0, p->x[i], p->y[i], p->z[i], hi, dens_visit, &c);
    } else {
        for (int64_t j = 0; j < p->n; ++j) dens_visit(j, &c);
    }
    double h3 = hi * hi * hi;
    *rho = 8.0 / (ORA_PI * h3) * (m[i] + c.sf);                     /* self: f(0) = 1 */
    *drho = -8.0 / (ORA_PI * h3 * hi) * (3.0 * m[i] + c.sg);        /* self: g(0) = 3 */
    *nw = (32.0 / 3.0) * (1.0 + c.sw);
    *dnw = -(32.0 / (3.0 * hi)) * c.sqdf;
    *nn = c.nn;
    *hash = c.hash;
}

static int check_set(const ora_pos* p, const double* h, int64_t nt, const int64_t* tgt) {
    if (p->n < 0 || !p->x || !p->y || !p->z || !(p->box > 0)) return ORA_E_ARG;
    if (h) for (int64_t i = 0; i < p->n; ++i)
        if (!(h[i] > 0) || !(h[i] < 0.5 * p->box)) return ORA_E_ARG;
    if (tgt) for (int64_t k = 0; k < nt; ++k) if (tgt[k] < 0 || tgt[k] >= p->n) return ORA_E_ARG;
    return ORA_OK;
}

/* targets == NULL: every particle.  Outputs are indexed by particle. */
int ora_density(int64_t n, const double* x, const double* y, const double* z, double box,
                const double* h, const double* m, int64_t nt, const int64_t* targets, int brute,
                double* rho, double* drho_dh, double* nw, double* dnw_dh, int64_t* nngb, uint64_t* hash) {
    ora_pos p = { n, x, y, z, box };
    int st = check_set(&p, h, nt, targets);
    if (st) return st;
    ora_grid g;
    if (!brute && (st = grid_build(&g, &p, h, 0))) return st;
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? targets[k] : k;
        density_one(&p, brute ? NULL : &g, m, i, h[i], &rho[i], &drho_dh[i], &nw[i], &dnw_dh[i],
                    &nngb[i], &hash[i]);
    }
    if (!brute) grid_free(&g);
    return ORA_OK;
}

/* ---------------------------------------------------------------------------
 * Smoothing-length solve: per particle, the h with |N_w(h) - target| <= tol.
 * N_w(h) = (32/3) sum_j f(r_ij/h) is continuous and non-decreasing in h and
 * strictly increasing once a neighbour is in range, so the root is unique.
 * Safeguarded Newton: keep a bracket [lo, hi]; take the Newton step unless it
 * leaves the bracket, leaves [h/2, 2h] or the slope is not positive; then
 * bisect (or double h while no upper end is known).
 * ------------------------------------------------------------------------- */
int ora_solve_h(int64_t n, const double* x, const double* y, const double* z, double box,
                const double* m, double* h, int64_t nt, const int64_t* targets, int brute,
                double target_nw, double tol, int max_iter, int32_t* iters, int64_t* n_unconverged) {
    ora_pos p = { n, x, y, z, box };
    int st = check_set(&p, h, nt, targets);
    if (st) return st;
    ora_grid g;
    if (!brute && (st = grid_build(&g, &p, NULL, 0))) return st;
    int64_t cnt = targets ? nt : n, bad = 0;
    const double hcap = 0.5 * box;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? targets[k] : k;
        double hi_ = h[i], lo = 0.0, up = INFINITY;
        int it = 0, ok = 0;
        for (; it < max_iter; ++it) {
            double rho, drho, nw, dnw;
            int64_t nn;
            uint64_t hs;
            density_one(&p, brute ? NULL : &g, m, i, hi_, &rho, &drho, &nw, &dnw, &nn, &hs);
            double err = nw - target_nw;
            if (fabs(err) <= tol) { ok = 1; break; }
            if (err < 0) lo = hi_; else up = hi_;
            double hn = (dnw > 0) ? hi_ - err / dnw : NAN;
            int bad_step = !(dnw > 0) || !(hn > lo) || !(hn < up) || !(hn >= 0.5 * hi_) || !(hn <= 2.0 * hi_);
            if (bad_step) hn = isinf(up) ? 2.0 * hi_ : 0.5 * (lo + up);
            if (hn >= hcap) hn = 0.5 * (hi_ + hcap);
            hi_ = hn;
        }
        h[i] = hi_;
        if (iters) iters[i] = it;
        if (!ok) bad += 1;
    }
    if (!brute) grid_free(&g);
    if (n_unconverged) *n_unconverged = bad;
    return bad ? ORA_E_NOCONV : ORA_OK;
}

/* ---------------------------------------------------------------------------
 * Ghost (per-particle equation of state between the two stages):
 *   P = (gamma-1) rho u,  c = sqrt(gamma (gamma-1) u),
 *   f = [1 + h/(3 rho) drho/dh]^-1,  A = f P / rho^2.
 * ------------------------------------------------------------------------- */
int ora_ghost(int64_t n, const double* h, const double* rho, const double* drho_dh, const double* u,
              double gamma, double* P, double* cs, double* fgrad, double* A) {
    if (n < 0) return ORA_E_ARG;
    for (int64_t i = 0; i < n; ++i) {
        double Pi = (gamma - 1.0) * rho[i] * u[i];
        double fi = 1.0 / (1.0 + h[i] / (3.0 * rho[i]) * drho_dh[i]);
        if (P) P[i] = Pi;
        if (cs) cs[i] = sqrt(gamma * (gamma - 1.0) * u[i]);
        if (fgrad) fgrad[i] = fi;
        if (A) A[i] = fi * Pi / (rho[i] * rho[i]);
    }
    return ORA_OK;
}

/* ---------------------------------------------------------------------------
 * Force stage (Section II, item 2): for each i, all j != i with
 * r_ij < max(h_i, h_j).  With G_i = grad_i W(r_ij, h_i), G_j =
 * grad_i W(r_ij, h_j), Gbar = (G_i + G_j)/2, w = v_ij.x_ij / r and
 * Pi_ij = -(alpha/2)(c_i + c_j - 3w) w / rhobar for w < 0 (else 0):
 *   a_i     = -sum_j m_j [A_i G_i + A_j G_j + Pi_ij Gbar]
 *   du_i/dt =  sum_j m_j [A_i v_ij.G_i + (1/2) Pi_ij v_ij.Gbar]
 *   vsig_i  =  max_j (c_i + c_j - 3 min(w, 0))
 *   S_i     =  sum_j m_j |A_i G_i + A_j G_j + Pi_ij Gbar|   (error scale)
 * ------------------------------------------------------------------------- */
typedef struct {
    const ora_pos* p;
    const double *h, *m, *vx, *vy, *vz, *rho, *A, *cs;
    double alpha;
    int64_t i;
    double ax, ay, az, du, vsig, S;
    int64_t nn;
    uint64_t hash;
} force_ctx;

static void force_visit(int64_t j, void* vctx) {
    force_ctx* c = (force_ctx*)vctx;
    int64_t i = c->i;
    if (j == i) return;
    const ora_pos* p = c->p;
    double dx = min_image(p->x[i] - p->x[j], p->box);
    double dy = min_image(p->y[i] - p->y[j], p->box);
    double dz = min_image(p->z[i] - p->z[j], p->box);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double hi = c->h[i], hj = c->h[j];
    if (!(r < (hi > hj ? hi : hj))) return;
    double ki = ora_gradW_factor(r, hi), kj = ora_gradW_factor(r, hj);
    double vxij = c->vx[i] - c->vx[j], vyij = c->vy[i] - c->vy[j], vzij = c->vz[i] - c->vz[j];
    double vdotx = vxij * dx + vyij * dy + vzij * dz;
    double w = vdotx / r;
    double visc = 0.0;
    if (w < 0.0) {
        double rhobar = 0.5 * (c->rho[i] + c->rho[j]);
        visc = -0.5 * c->alpha * (c->cs[i] + c->cs[j] - 3.0 * w) * w / rhobar;
    }
    /* vector term A_i G_i + A_j G_j + Pi Gbar = x_ij * s */
    double s = c->A[i] * ki + c->A[j] * kj + visc * 0.5 * (ki + kj);
    double mj = c->m[j];
    c->ax -= mj * s * dx;
    c->ay -= mj * s * dy;
    c->az -= mj * s * dz;
    c->du += mj * vdotx * (c->A[i] * ki + 0.5 * visc * 0.5 * (ki + kj));
    double vs = c->cs[i] + c->cs[j] - 3.0 * (w < 0.0 ? w : 0.0);
    if (vs > c->vsig) c->vsig = vs;
    c->S += mj * fabs(s) * r;
    c->nn += 1;
    c->hash += ora_mix((uint64_t)j);
}

int ora_force(int64_t n, const double* x, const double* y, const double* z, double box,
              const double* h, const double* m, const double* vx, const double* vy, const double* vz,
              const double* u, const double* rho, const double* drho_dh, double gamma, double alpha,
              int64_t nt, const int64_t* targets, int brute,
              double* ax, double* ay, double* az, double* dudt, double* vsig, double* S,
              int64_t* nforce, uint64_t* hash) {
    ora_pos p = { n, x, y, z, box };
    int st = check_set(&p, h, nt, targets);
    if (st) return st;
    double* A = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* cs = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!A || !cs) { free(A); free(cs); return ORA_E_MEM; }
    ora_ghost(n, h, rho, drho_dh, u, gamma, NULL, cs, NULL, A);
    ora_grid g;
    if (!brute && (st = grid_build(&g, &p, h, 1))) { free(A); free(cs); return st; }
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? targets[k] : k;
        force_ctx c = { &p, h, m, vx, vy, vz, rho, A, cs, alpha, i, 0, 0, 0, 0, 0, 0, 0, 0 };
        if (brute) {
            for (int64_t j = 0; j < n; ++j) force_visit(j, &c);
        } else {
            for (int cl = 0; cl < g.ncls; ++cl) {
                double R = h[i] > g.hmax[cl] ? h[i] : g.hmax[cl];
                grid_query(&g, &p, cl, x[i], y[i], z[i], R, force_visit, &c);
            }
        }
        ax[i] = c.ax; ay[i] = c.ay; az[i] = c.az;
        dudt[i] = c.du; vsig[i] = c.vsig; S[i] = c.S;
        nforce[i] = c.nn; hash[i] = c.hash;
    }
    if (!brute) grid_free(&g);
    free(A); free(cs);
    return ORA_OK;
}

/* Global FP64 sums: momentum M = sum m a, energy rate
 * E = sum m (v.a + du/dt) and the bound scale sum m S. out[0..4] =
 * Mx, My, Mz, E, scale. */
int ora_sums(int64_t n, const double* m, const double* vx, const double* vy, const double* vz,
             const double* ax, const double* ay, const double* az, const double* dudt,
             const double* S, double* out) {
    double Mx = 0, My = 0, Mz = 0, E = 0, sc = 0;
    for (int64_t i = 0; i < n; ++i) {
        Mx += m[i] * ax[i]; My += m[i] * ay[i]; Mz += m[i] * az[i];
        E += m[i] * (vx[i] * ax[i] + vy[i] * ay[i] + vz[i] * az[i] + dudt[i]);
        sc += m[i] * S[i];
    }
    out[0] = Mx; out[1] = My; out[2] = Mz; out[3] = E; out[4] = sc;
    return ORA_OK;
}

/* Per particle: 1 if some j has r_ij within rel of h_i or of h_j (a pair
 * whose membership in the density or force set would hinge on rounding). */
typedef struct { const ora_pos* p; const double* h; int64_t i; double rel; int flag; } tie_ctx;

static void tie_visit(int64_t j, void* vctx) {
    tie_ctx* c = (tie_ctx*)vctx;
    if (j == c->i) return;
    const ora_pos* p = c->p;
    double dx = min_image(p->x[c->i] - p->x[j], p->box);
    double dy = min_image(p->y[c->i] - p->y[j], p->box);
    double dz = min_image(p->z[c->i] - p->z[j], p->box);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double a = c->h[c->i], b = c->h[j];
    if (fabs(r / a - 1.0) < c->rel || fabs(r / b - 1.0) < c->rel) c->flag = 1;
}

int ora_near_cutoff(int64_t n, const double* x, const double* y, const double* z, double box,
                    const double* h, double rel, int brute, int64_t nt, const int64_t* targets, uint8_t* flag) {
    ora_pos p = { n, x, y, z, box };
    int st = check_set(&p, h, nt, targets);
    if (st) return st;
    ora_grid g;
    if (!brute && (st = grid_build(&g, &p, h, 1))) return st;
    int64_t cnt = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = targets ? targets[k] : k;
        tie_ctx c = { &p, h, i, rel, 0 };
        if (brute) {
            for (int64_t j = 0; j < n; ++j) tie_visit(j, &c);
        } else {
            for (int cl = 0; cl < g.ncls; ++cl) {
                double R = (h[i] > g.hmax[cl] ? h[i] : g.hmax[cl]) * (1.0 + 2.0 * rel);
                grid_query(&g, &p, cl, x[i], y[i], z[i], R, tie_visit, &c);
            }
        }
        flag[i] = (uint8_t)c.flag;
    }
    if (!brute) grid_free(&g);
    return ORA_OK;
}

/* Mark every particle that is a force neighbour (r < max(h_i, h_j)) of one
 * of the targets, and the targets themselves (to know whose densities a
 * sampled force evaluation needs). */
typedef struct { const ora_pos* p; const double* h; int64_t i; uint8_t* mark; } nb_ctx;

static void nb_visit(int64_t j, void* vctx) {
    nb_ctx* c = (nb_ctx*)vctx;
    const ora_pos* p = c->p;
    double dx = min_image(p->x[c->i] - p->x[j], p->box);
    double dy = min_image(p->y[c->i] - p->y[j], p->box);
    double dz = min_image(p->z[c->i] - p->z[j], p->box);
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double a = c->h[c->i], b = c->h[j];
    if (r < (a > b ? a : b)) c->mark[j] = 1;
}

int ora_force_neighbours(int64_t n, const double* x, const double* y, const double* z, double box,
                         const double* h, int64_t nt, const int64_t* targets, uint8_t* mark) {
    ora_pos p = { n, x, y, z, box };
    int st = check_set(&p, h, nt, targets);
    if (st) return st;
    if (!targets) return ORA_E_ARG;
    ora_grid g;
    if ((st = grid_build(&g, &p, h, 1))) return st;
    /* serial over targets: marks are written by many targets */
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = targets[k];
        nb_ctx c = { &p, h, i, mark };
        mark[i] = 1;
        for (int cl = 0; cl < g.ncls; ++cl) {
            double R = h[i] > g.hmax[cl] ? h[i] : g.hmax[cl];
            grid_query(&g, &p, cl, x[i], y[i], z[i], R, nb_visit, &c);
        }
    }
    grid_free(&g);
    return ORA_OK;
}

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
