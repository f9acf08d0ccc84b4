/*
 * FP64 CPU oracle for the explicit finite-difference star-stencil sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links, imports or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or table with the GPU path.
 *
 * What it computes (the plain definitions, in FP64, with straightforward
 * loops; OpenMP only splits the outermost loop):
 *
 *   Fields are dense C-order buffers whose bounds include the halo, as the
 *   stencil dialect's field type carries its bounds (Section 4.1).  A grid has
 *   ndim active axes (the last ndim of z, y, x); the interior of an active
 *   axis is [h, h + n) and the buffer extent is n + 2h.
 *
 *   Star operator (stencil.apply reading stencil.access offsets along the
 *   axes only, Section 4.1; Figure "stencil_intro" for the 1D 3-point case):
 *       (L u)_i = D c_0 u_i + sum_{axes d} sum_{k=1..r} c_k (u_{i+k e_d} + u_{i-k e_d})
 *   Heat / Jacobi (the Devito heat listing, u.dt = a * laplace(u) solved for
 *   u.forward, Section 5.1), with the weights already scaled by a dt / h^2:
 *       u^{n+1} = u^n + L u^n
 *   Acoustic wave, second order in time (Section 6.1):
 *       u^{n+1} = 2 u^n - u^{n-1} + beta .* (L u^n),   beta = (dt v / h)^2
 *   then sources add their per-step amount and receivers sample u^{n+1}.
 *
 *   Halo exchange declarations (the dmp.exchange attribute, Section 4.2): a
 *   receive box [at, at+size), a send box shifted by the source offset and the
 *   relative rank it goes to.  Faces only for the star; the box form adds the
 *   edges and corners a stencil with diagonal offsets reads.
 *
 *   A stencil program (several stencil.apply results over several fields,
 *   fused into one region as Section 6.2 describes for PW advection): each
 *   output is a sum, in program order, of terms c * f(i + o) or
 *   c * f(i + o) * g(i + o') over input fields f, g at arbitrary offsets
 *   within the halo.
 *
 *   A Piacsek-Williams-style advection (Section 6.2 names the scheme; no
 *   formulas are printed): the flux-form, centred advection of the velocity
 *   (u, v, w) on a staggered C grid, written out directly in
 *   orc_pw_advection below.
 *
 *   Off-grid points (Devito's sparse functions, Section 5.1, at real
 *   positions): multilinear interpolation over the 2^ndim corners of the
 *   grid cell holding the position; a source adds weight * amplitude at each
 *   corner, a receiver records the weighted sum of the corner values.
 *
 *   Absorbing layer: the wave equation with a damping term, m u_tt + eta u_t
 *   = laplace(u) / h^2 + q, central differences in time.  With the
 *   dimensionless gamma = eta dt / (2 m) per point:
 *       u^{n+1} = (2 u^n - (1 - gamma) u^{n-1} + beta .* (L u^n)) / (1 + gamma)
 *   and the sources added after the update as in the undamped step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)

/* must match the layout the Python wrapper declares */
typedef struct {
    int64_t at[3];
    int64_t size[3];
    int64_t src_offset[3];
    int32_t to[3];
    int32_t pad_;
} orc_exchange;

typedef struct {
    int ndim;
    int h;
    int64_t n[3]; /* interior extents, internal axes (z, y, x); 1 when inactive */
    int64_t e[3]; /* buffer extents */
    int64_t s[3]; /* strides in elements */
    int64_t total;
} og;

static int og_init(og* g, int ndim, const int64_t* shape, int halo) {
    if (ndim < 1 || ndim > 3 || halo < 0) return ORC_EINVAL;
    g->ndim = ndim;
    g->h = halo;
    for (int a = 0; a < 3; a++) {
        int active = a >= 3 - ndim;
        g->n[a] = active ? shape[a - (3 - ndim)] : 1;
        if (g->n[a] < 0) return ORC_EINVAL;
        g->e[a] = active ? g->n[a] + 2 * halo : 1;
    }
    g->s[2] = 1;
    g->s[1] = g->e[2];
    g->s[0] = g->e[1] * g->e[2];
    g->total = g->e[0] * g->e[1] * g->e[2];
    return ORC_OK;
}

static int og_active(const og* g, int a) { return a >= 3 - g->ndim; }

/* interior lower bound on internal axis a */
static int64_t og_lo(const og* g, int a) { return og_active(g, a) ? g->h : 0; }

/* buffer offset of an interior position given as ndim coordinates (C order) */
static int64_t og_pos(const og* g, const int64_t* p3) {
    int64_t off = 0;
    for (int a = 0; a < 3; a++) {
        int64_t c = og_active(g, a) ? p3[a - (3 - g->ndim)] + g->h : 0;
        off += c * g->s[a];
    }
    return off;
}

static int og_pos_ok(const og* g, const int64_t* p3) {
    for (int i = 0; i < g->ndim; i++) {
        int a = i + 3 - g->ndim;
        if (p3[i] < 0 || p3[i] >= g->n[a]) return 0;
    }
    return 1;
}

/* (L u) at buffer offset p */
static double star_at(const og* g, int radius, const double* c, const double* u, int64_t p) {
    double acc = (double)g->ndim * c[0] * u[p];
    for (int a = 0; a < 3; a++) {
        if (!og_active(g, a)) continue;
        for (int k = 1; k <= radius; k++)
            acc += c[k] * (u[p + k * g->s[a]] + u[p - k * g->s[a]]);
    }
    return acc;
}

static int check_common(const og* g, int radius) {
    if (radius < 1 || radius > g->h) return ORC_EINVAL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* star operator, heat sweep                                                  */
/* ------------------------------------------------------------------------ */

int orc_star(int ndim, const int64_t* shape, int halo, int radius, const double* c,
             const double* u, double* out) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius)) return ORC_EINVAL;
    int64_t lz = og_lo(&g, 0), ly = og_lo(&g, 1), lx = og_lo(&g, 2);
#pragma omp parallel for schedule(static)
    for (int64_t z = lz; z < lz + g.n[0]; z++)
        for (int64_t y = ly; y < ly + g.n[1]; y++)
            for (int64_t x = lx; x < lx + g.n[2]; x++) {
                int64_t p = z * g.s[0] + y * g.s[1] + x;
                out[p] = star_at(&g, radius, c, u, p);
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* exchange declarations, pack / unpack                                       */
/* ------------------------------------------------------------------------ */

/*
 * For each active axis and each side with a neighbour (always, when the
 * decomposition is periodic), one exchange: the halo slab of thickness
 * `radius` on that side is received, and the interior slab of the same size
 * on the same face, shifted inwards by `radius`, is sent.
 * Low side: at = h - r, offset +r, to = -1.  High side: at = h + n,
 * offset -r, to = +1.  The other axes span the interior only (no corners).
 */
int orc_exchanges(int ndim, const int64_t* shape, int halo, int radius, const int32_t* grid,
                  const int32_t* coord, int periodic, orc_exchange* out, int* count) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || !count) return ORC_EINVAL;
    int cap = *count, k = 0;
    for (int i = 0; i < ndim; i++) {
        if (grid[i] < 1 || coord[i] < 0 || coord[i] >= grid[i]) return ORC_EINVAL;
        for (int side = 0; side < 2; side++) {
            int has = periodic || (side == 0 ? coord[i] > 0 : coord[i] < grid[i] - 1);
            if (!has) continue;
            if (k < cap && out) {
                orc_exchange* x = &out[k];
                memset(x, 0, sizeof(*x));
                for (int j = 0; j < ndim; j++) {
                    x->at[j] = halo;
                    x->size[j] = shape[j];
                }
                x->size[i] = radius;
                if (side == 0) {
                    x->at[i] = halo - radius;
                    x->src_offset[i] = radius;
                    x->to[i] = -1;
                } else {
                    x->at[i] = halo + shape[i];
                    x->src_offset[i] = -radius;
                    x->to[i] = 1;
                }
            }
            k++;
        }
    }
    *count = k;
    return (out && k > cap) ? ORC_EINVAL : ORC_OK;
}

static int64_t ex_elems(const og* g, const orc_exchange* x) {
    int64_t c = 1;
    for (int i = 0; i < g->ndim; i++) c *= x->size[i];
    return c;
}

static int ex_box_ok(const og* g, const int64_t* at, const int64_t* size) {
    for (int i = 0; i < g->ndim; i++) {
        int a = i + 3 - g->ndim;
        if (size[i] < 0 || at[i] < 0 || at[i] + size[i] > g->e[a]) return 0;
    }
    return 1;
}

/* copy box [lo, lo+size) of `field` to / from the contiguous C-order `buf` */
static void box_copy(const og* g, double* field, const int64_t* lo, const int64_t* size, double* buf,
                     int to_buf) {
    int64_t L[3] = {0, 0, 0}, S[3] = {1, 1, 1};
    for (int i = 0; i < g->ndim; i++) {
        L[i + 3 - g->ndim] = lo[i];
        S[i + 3 - g->ndim] = size[i];
    }
    int64_t q = 0;
    for (int64_t z = 0; z < S[0]; z++)
        for (int64_t y = 0; y < S[1]; y++)
            for (int64_t x = 0; x < S[2]; x++, q++) {
                int64_t p = (L[0] + z) * g->s[0] + (L[1] + y) * g->s[1] + (L[2] + x);
                if (to_buf)
                    buf[q] = field[p];
                else
                    field[p] = buf[q];
            }
}

int orc_pack(int ndim, const int64_t* shape, int halo, const double* field, const orc_exchange* ex,
             int n, double* buf) {
    og g;
    if (og_init(&g, ndim, shape, halo)) return ORC_EINVAL;
    int64_t off = 0;
    for (int k = 0; k < n; k++) {
        int64_t lo[3];
        for (int i = 0; i < 3; i++) lo[i] = ex[k].at[i] + ex[k].src_offset[i];
        if (!ex_box_ok(&g, lo, ex[k].size)) return ORC_EINVAL;
        box_copy(&g, (double*)field, lo, ex[k].size, buf + off, 1);
        off += ex_elems(&g, &ex[k]);
    }
    return ORC_OK;
}

int orc_unpack(int ndim, const int64_t* shape, int halo, double* field, const orc_exchange* ex,
               int n, const double* buf) {
    og g;
    if (og_init(&g, ndim, shape, halo)) return ORC_EINVAL;
    int64_t off = 0;
    for (int k = 0; k < n; k++) {
        if (!ex_box_ok(&g, ex[k].at, ex[k].size)) return ORC_EINVAL;
        box_copy(&g, field, ex[k].at, ex[k].size, (double*)buf + off, 0);
        off += ex_elems(&g, &ex[k]);
    }
    return ORC_OK;
}

/*
 * Periodic boundary on one rank: every exchange's neighbour is the rank
 * itself, so the halo received through the exchange with relative rank t is
 * what the exchange with relative rank -t sends.
 */
static int periodic_refresh(const og* g, const int64_t* shape, int radius, double* u) {
    int32_t grid[3] = {1, 1, 1}, coord[3] = {0, 0, 0};
    orc_exchange ex[6];
    int n = 6;
    int rc = orc_exchanges(g->ndim, shape, g->h, radius, grid, coord, 1, ex, &n);
    if (rc) return rc;
    int64_t off[7];
    off[0] = 0;
    for (int k = 0; k < n; k++) off[k + 1] = off[k] + ex_elems(g, &ex[k]);
    double* buf = (double*)malloc(sizeof(double) * (size_t)(off[n] > 0 ? off[n] : 1));
    if (!buf) return ORC_ENOMEM;
    rc = orc_pack(g->ndim, shape, g->h, u, ex, n, buf);
    for (int k = 0; k < n && !rc; k++) {
        int partner = -1;
        for (int j = 0; j < n; j++) {
            int match = 1;
            for (int i = 0; i < g->ndim; i++) match &= ex[j].to[i] == -ex[k].to[i];
            if (match) partner = j;
        }
        if (partner < 0) {
            rc = ORC_EINVAL;
            break;
        }
        rc = orc_unpack(g->ndim, shape, g->h, u, &ex[k], 1, buf + off[partner]);
    }
    free(buf);
    return rc;
}

int orc_heat_run(int ndim, const int64_t* shape, int halo, int radius, const double* c, int periodic,
                 double* u, int64_t nsteps) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || nsteps < 0) return ORC_EINVAL;
    double* v = (double*)malloc(sizeof(double) * (size_t)g.total);
    if (!v) return ORC_ENOMEM;
    memcpy(v, u, sizeof(double) * (size_t)g.total);
    int64_t lz = og_lo(&g, 0), ly = og_lo(&g, 1), lx = og_lo(&g, 2);
    for (int64_t t = 0; t < nsteps; t++) {
        if (periodic) {
            int rc = periodic_refresh(&g, shape, radius, u);
            if (rc) {
                free(v);
                return rc;
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t z = lz; z < lz + g.n[0]; z++)
            for (int64_t y = ly; y < ly + g.n[1]; y++)
                for (int64_t x = lx; x < lx + g.n[2]; x++) {
                    int64_t p = z * g.s[0] + y * g.s[1] + x;
                    v[p] = u[p] + star_at(&g, radius, c, u, p);
                }
        /* the new level becomes the current one; v's halo equals u's */
        memcpy(u, v, sizeof(double) * (size_t)g.total);
    }
    free(v);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* acoustic wave, second order in time                                        */
/* ------------------------------------------------------------------------ */

static int wave_step(const og* g, const int64_t* shape, int radius, const double* c, int periodic,
                     const double* beta, double* un, const double* unm1, double* out) {
    if (periodic) {
        int rc = periodic_refresh(g, shape, radius, un);
        if (rc) return rc;
    }
    int64_t lz = og_lo(g, 0), ly = og_lo(g, 1), lx = og_lo(g, 2);
#pragma omp parallel for schedule(static)
    for (int64_t z = lz; z < lz + g->n[0]; z++)
        for (int64_t y = ly; y < ly + g->n[1]; y++)
            for (int64_t x = lx; x < lx + g->n[2]; x++) {
                int64_t p = z * g->s[0] + y * g->s[1] + x;
                out[p] = 2.0 * un[p] - unm1[p] + beta[p] * star_at(g, radius, c, un, p);
            }
    return ORC_OK;
}

static int pos_list_ok(const og* g, int64_t n, const int64_t* pos) {
    if (n < 0 || (n > 0 && !pos)) return 0;
    for (int64_t i = 0; i < n; i++)
        if (!og_pos_ok(g, pos + 3 * i)) return 0;
    return 1;
}

/*
 * nsteps leapfrog steps from (u_n, u_nm1) = (u^0, u^{-1}).  After the sweep
 * of step t the sources add src_amp[t][s] at their points and the receivers
 * record traces[t][r] = u^{t+1} at theirs.  On return u_n = u^N and
 * u_nm1 = u^{N-1}.  Positions are interior coordinates, 3 slots per point
 * (the first ndim used, C order).
 */
int orc_wave_run(int ndim, const int64_t* shape, int halo, int radius, const double* c, int periodic,
                 const double* beta, double* u_n, double* u_nm1, int64_t nsteps, int64_t nsrc,
                 const int64_t* src, const double* src_amp, int64_t nrec, const int64_t* rec,
                 double* traces) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || nsteps < 0) return ORC_EINVAL;
    if (!pos_list_ok(&g, nsrc, src) || !pos_list_ok(&g, nrec, rec)) return ORC_EINVAL;
    if ((nsrc > 0 && !src_amp) || (nrec > 0 && !traces)) return ORC_EINVAL;
    double* a = u_n;   /* u^t */
    double* b = u_nm1; /* u^{t-1}, overwritten by u^{t+1} */
    for (int64_t t = 0; t < nsteps; t++) {
        int rc = wave_step(&g, shape, radius, c, periodic, beta, a, b, b);
        if (rc) return rc;
        for (int64_t s = 0; s < nsrc; s++) b[og_pos(&g, src + 3 * s)] += src_amp[t * nsrc + s];
        for (int64_t r = 0; r < nrec; r++) traces[t * nrec + r] = b[og_pos(&g, rec + 3 * r)];
        double* tmp = a;
        a = b;
        b = tmp;
    }
    if (a != u_n) { /* odd number of steps: the newest level sits in u_nm1 */
        size_t bytes = sizeof(double) * (size_t)g.total;
        double* tmp = (double*)malloc(bytes);
        if (!tmp) return ORC_ENOMEM;
        memcpy(tmp, a, bytes);     /* a is the u_nm1 buffer and holds u^N */
        memcpy(u_nm1, u_n, bytes); /* u_n held u^{N-1} */
        memcpy(u_n, tmp, bytes);
        free(tmp);
    }
    return ORC_OK;
}

/*
 * Discrete adjoint of the leapfrog recurrence with respect to the squared
 * slowness m (beta = dt^2 / (h^2 m)).  Writing the step as
 *     m (u^{n+1} - 2u^n + u^{n-1}) - (dt^2/h^2) L u^n - dt^2 q^n = 0,
 * whose Jacobian blocks are symmetric (L is symmetric for the star with a
 * zero halo), the adjoint field obeys, for k = N..1 with lam^N = lam^{N+1} = 0,
 *     lam^{k-1} = 2 lam^k - lam^{k+1} + beta .* (L lam^k) + w_r r^k at receivers,
 * which is the forward sweep run backwards in time with the residuals
 * injected at the receivers (w_r = dt^2 v_r^2 for the L2 misfit).
 * `adj_step_out` receives lam^{k-1} for k = N..1 at the probe points:
 * probe_out[(k-1)][p].
 */
static int adjoint_core(const og* g, const int64_t* shape, int radius, const double* c,
                        const double* beta, int64_t nsteps, int64_t nrec, const int64_t* rec,
                        const double* rec_w, const double* resid, int64_t nprobe, const int64_t* probe,
                        double* probe_out, const double* states, double gscale, double* grad) {
    double* a = (double*)calloc((size_t)g->total, sizeof(double)); /* lam^k */
    double* b = (double*)calloc((size_t)g->total, sizeof(double)); /* lam^{k+1} -> lam^{k-1} */
    if (!a || !b) {
        free(a);
        free(b);
        return ORC_ENOMEM;
    }
    int64_t lz = og_lo(g, 0), ly = og_lo(g, 1), lx = og_lo(g, 2);
    for (int64_t k = nsteps; k >= 1; k--) {
        wave_step(g, shape, radius, c, 0, beta, a, b, b);
        for (int64_t r = 0; r < nrec; r++)
            b[og_pos(g, rec + 3 * r)] += rec_w[r] * resid[(k - 1) * nrec + r];
        for (int64_t p = 0; p < nprobe; p++) probe_out[(k - 1) * nprobe + p] = b[og_pos(g, probe + 3 * p)];
        if (states && grad) {
            /* states holds u^{-1}, u^0, ..., u^N; D^{k-1} = u^k - 2u^{k-1} + u^{k-2} */
            const double* up = states + (size_t)(k + 1) * (size_t)g->total;
            const double* uc = states + (size_t)(k) * (size_t)g->total;
            const double* um = states + (size_t)(k - 1) * (size_t)g->total;
#pragma omp parallel for schedule(static)
            for (int64_t z = lz; z < lz + g->n[0]; z++)
                for (int64_t y = ly; y < ly + g->n[1]; y++)
                    for (int64_t x = lx; x < lx + g->n[2]; x++) {
                        int64_t p = z * g->s[0] + y * g->s[1] + x;
                        int64_t q = ((z - lz) * g->n[1] + (y - ly)) * g->n[2] + (x - lx);
                        grad[q] += gscale * b[p] * (up[p] - 2.0 * uc[p] + um[p]);
                    }
        }
        double* tmp = a;
        a = b;
        b = tmp;
    }
    free(a);
    free(b);
    return ORC_OK;
}

int orc_wave_adjoint(int ndim, const int64_t* shape, int halo, int radius, const double* c,
                     const double* beta, int64_t nsteps, int64_t nrec, const int64_t* rec,
                     const double* rec_w, const double* resid, int64_t nprobe, const int64_t* probe,
                     double* probe_out) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || nsteps < 0) return ORC_EINVAL;
    if (!pos_list_ok(&g, nrec, rec) || !pos_list_ok(&g, nprobe, probe)) return ORC_EINVAL;
    if ((nrec > 0 && (!rec_w || !resid)) || (nprobe > 0 && !probe_out)) return ORC_EINVAL;
    return adjoint_core(&g, shape, radius, c, beta, nsteps, nrec, rec, rec_w, resid, nprobe, probe,
                        probe_out, NULL, 0.0, NULL);
}

/*
 * Misfit J = 1/2 sum_{n=1..N} sum_r (d^n_r - dobs^n_r)^2 and its gradient
 *     g = gscale * sum_{n=0..N-1} lam^n .* (u^{n+1} - 2u^n + u^{n-1}),
 * gscale = -1/dt^2 for the gradient with respect to m.  The forward keeps
 * every level in memory (the oracle is for small grids).  traces[n-1][r]
 * receives d^n; grad is interior-shaped and dense.
 */
int orc_wave_gradient(int ndim, const int64_t* shape, int halo, int radius, const double* c,
                      const double* beta, int64_t nsteps, int64_t nsrc, const int64_t* src,
                      const double* src_amp, int64_t nrec, const int64_t* rec, const double* dobs,
                      const double* rec_w, double gscale, double* traces, double* misfit,
                      double* grad) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || nsteps < 0) return ORC_EINVAL;
    if (!pos_list_ok(&g, nsrc, src) || !pos_list_ok(&g, nrec, rec)) return ORC_EINVAL;
    if ((nsrc > 0 && !src_amp) || (nrec > 0 && (!dobs || !rec_w || !traces)) || !grad || !misfit)
        return ORC_EINVAL;
    size_t T = (size_t)g.total;
    double* states = (double*)calloc(T * (size_t)(nsteps + 2), sizeof(double));
    double* resid = (double*)calloc((size_t)(nsteps * nrec + 1), sizeof(double));
    if (!states || !resid) {
        free(states);
        free(resid);
        return ORC_ENOMEM;
    }
    /* states[0] = u^{-1} = 0, states[1] = u^0 = 0 */
    for (int64_t t = 0; t < nsteps; t++) {
        double* um = states + (size_t)t * T;
        double* uc = states + (size_t)(t + 1) * T;
        double* up = states + (size_t)(t + 2) * T;
        wave_step(&g, shape, radius, c, 0, beta, uc, um, up);
        for (int64_t s = 0; s < nsrc; s++) up[og_pos(&g, src + 3 * s)] += src_amp[t * nsrc + s];
        for (int64_t r = 0; r < nrec; r++) traces[t * nrec + r] = up[og_pos(&g, rec + 3 * r)];
    }
    double J = 0.0;
    for (int64_t i = 0; i < nsteps * nrec; i++) {
        resid[i] = traces[i] - dobs[i];
        J += 0.5 * resid[i] * resid[i];
    }
    *misfit = J;
    memset(grad, 0, sizeof(double) * (size_t)(g.n[0] * g.n[1] * g.n[2]));
    int rc = adjoint_core(&g, shape, radius, c, beta, nsteps, nrec, rec, rec_w, resid, 0, NULL, NULL,
                          states, gscale, grad);
    free(states);
    free(resid);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* box exchanges: faces, edges and corners                                    */
/* ------------------------------------------------------------------------ */

/* Every neighbour direction d in {-1, 0, 1}^ndim other than 0, in C order
 * (the first axis slowest, -1 before 0 before +1).  Per axis: d = -1 gives
 * at = h - r, size r, offset +r; d = 0 the interior [h, h + n) and offset 0;
 * d = +1 at = h + n, size r, offset -r.  A direction exists when every axis
 * with d != 0 has that neighbour (or the grid is periodic). */
int orc_exchanges_box(int ndim, const int64_t* shape, int halo, int radius, const int32_t* grid,
                      const int32_t* coord, int periodic, orc_exchange* out, int* count) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || !count) return ORC_EINVAL;
    for (int i = 0; i < ndim; i++)
        if (grid[i] < 1 || coord[i] < 0 || coord[i] >= grid[i]) return ORC_EINVAL;
    int cap = *count, k = 0;
    int ndir = 1;
    for (int i = 0; i < ndim; i++) ndir *= 3;
    for (int code = 0; code < ndir; code++) {
        int d[3] = {0, 0, 0}, rem = code, zero = 1, has = 1;
        for (int i = ndim - 1; i >= 0; i--) {
            d[i] = rem % 3 - 1;
            rem /= 3;
        }
        for (int i = 0; i < ndim; i++) {
            if (d[i] != 0) zero = 0;
            if (d[i] < 0 && !periodic && coord[i] == 0) has = 0;
            if (d[i] > 0 && !periodic && coord[i] == grid[i] - 1) has = 0;
        }
        if (zero || !has) continue;
        if (k < cap && out) {
            orc_exchange* x = &out[k];
            memset(x, 0, sizeof(*x));
            for (int i = 0; i < ndim; i++) {
                if (d[i] < 0) {
                    x->at[i] = halo - radius;
                    x->size[i] = radius;
                    x->src_offset[i] = radius;
                } else if (d[i] > 0) {
                    x->at[i] = halo + shape[i];
                    x->size[i] = radius;
                    x->src_offset[i] = -radius;
                } else {
                    x->at[i] = halo;
                    x->size[i] = shape[i];
                }
                x->to[i] = d[i];
            }
        }
        k++;
    }
    *count = k;
    return (out && k > cap) ? ORC_EINVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* stencil programs                                                           */
/* ------------------------------------------------------------------------ */

/* must match the layout the Python wrapper declares */
typedef struct {
    int32_t out;
    int32_t nfac;      /* 1 or 2 */
    int32_t in[2];
    int32_t off[2][3]; /* offsets per internal axis (z, y, x) */
    double coeff;
} orc_term;

/* out[o] on the interior: the terms of output o summed in program order,
 * each term coeff * in[a](i + off_a) (* in[b](i + off_b)).  Halos of the
 * outputs are left as they are. */
int orc_program(int ndim, const int64_t* shape, int halo, int nin, const double* const* ins, int nout,
                double* const* outs, int nterms, const orc_term* terms) {
    og g;
    if (og_init(&g, ndim, shape, halo) || nin < 1 || nout < 1 || nterms < 0) return ORC_EINVAL;
    for (int t = 0; t < nterms; t++) {
        const orc_term* T = &terms[t];
        if (T->out < 0 || T->out >= nout || T->nfac < 1 || T->nfac > 2) return ORC_EINVAL;
        for (int f = 0; f < T->nfac; f++) {
            if (T->in[f] < 0 || T->in[f] >= nin) return ORC_EINVAL;
            for (int a = 0; a < 3; a++) {
                int o = T->off[f][a];
                if (!og_active(&g, a) && o != 0) return ORC_EINVAL;
                if (o < -halo || o > halo) return ORC_EINVAL;
            }
        }
    }
    const int64_t lo0 = og_lo(&g, 0), lo1 = og_lo(&g, 1), lo2 = og_lo(&g, 2);
#pragma omp parallel for schedule(static)
    for (int64_t z = lo0; z < lo0 + g.n[0]; z++)
        for (int64_t y = lo1; y < lo1 + g.n[1]; y++)
            for (int64_t x = lo2; x < lo2 + g.n[2]; x++) {
                const int64_t p = z * g.s[0] + y * g.s[1] + x;
                for (int o = 0; o < nout; o++) {
                    double acc = 0.0;
                    for (int t = 0; t < nterms; t++) {
                        const orc_term* T = &terms[t];
                        if (T->out != o) continue;
                        double v = T->coeff;
                        for (int f = 0; f < T->nfac; f++) {
                            const int64_t q = p + T->off[f][0] * g.s[0] + T->off[f][1] * g.s[1] + T->off[f][2];
                            v *= ins[T->in[f]][q];
                        }
                        acc += v;
                    }
                    outs[o][p] = acc;
                }
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* flux-form centred advection on a C grid                                    */
/* ------------------------------------------------------------------------ */

/* Velocity on a staggered (Arakawa C) grid: u[k][j][i] lives at the x face
 * (i + 1/2, j, k), v[k][j][i] at (i, j + 1/2, k), w[k][j][i] at
 * (i, j, k + 1/2).  The advective tendency of each component is minus the
 * divergence of its momentum flux, with every product formed from two-point
 * averages onto the flux position:
 *   su = -[ dx( (u^x)^2 ) + dy( v^x u^y ) + dz( w^x u^z ) ]
 *   sv = -[ dx( u^y v^x ) + dy( (v^y)^2 ) + dz( w^y v^z ) ]
 *   sw = -[ dx( u^z w^x ) + dy( v^z w^y ) + dz( (w^z)^2 ) ]
 * where q^a is the average of q with its neighbour along a (towards + for
 * the flux on the high face of the cell, towards - for the low face) and
 * da(F) = (F_high - F_low) / h_a.  Written out point by point below. */
int orc_pw_advection(const int64_t* shape, int halo, const double* u, const double* v, const double* w,
                     double dx, double dy, double dz, double* su, double* sv, double* sw) {
    og g;
    if (og_init(&g, 3, shape, halo) || halo < 1) return ORC_EINVAL;
    const int64_t X = 1, Y = g.s[1], Z = g.s[0];
#pragma omp parallel for schedule(static)
    for (int64_t k = halo; k < halo + g.n[0]; k++)
        for (int64_t j = halo; j < halo + g.n[1]; j++)
            for (int64_t i = halo; i < halo + g.n[2]; i++) {
                const int64_t p = k * Z + j * Y + i * X;
                /* u at (i+1/2, j, k) */
                {
                    const double fxh = 0.5 * (u[p] + u[p + X]), fxl = 0.5 * (u[p - X] + u[p]);
                    const double vyh = 0.5 * (v[p] + v[p + X]), uyh = 0.5 * (u[p] + u[p + Y]);
                    const double vyl = 0.5 * (v[p - Y] + v[p - Y + X]), uyl = 0.5 * (u[p - Y] + u[p]);
                    const double wzh = 0.5 * (w[p] + w[p + X]), uzh = 0.5 * (u[p] + u[p + Z]);
                    const double wzl = 0.5 * (w[p - Z] + w[p - Z + X]), uzl = 0.5 * (u[p - Z] + u[p]);
                    su[p] = -((fxh * fxh - fxl * fxl) / dx + (vyh * uyh - vyl * uyl) / dy + (wzh * uzh - wzl * uzl) / dz);
                }
                /* v at (i, j+1/2, k) */
                {
                    const double uxh = 0.5 * (u[p] + u[p + Y]), vxh = 0.5 * (v[p] + v[p + X]);
                    const double uxl = 0.5 * (u[p - X] + u[p - X + Y]), vxl = 0.5 * (v[p - X] + v[p]);
                    const double fyh = 0.5 * (v[p] + v[p + Y]), fyl = 0.5 * (v[p - Y] + v[p]);
                    const double wzh = 0.5 * (w[p] + w[p + Y]), vzh = 0.5 * (v[p] + v[p + Z]);
                    const double wzl = 0.5 * (w[p - Z] + w[p - Z + Y]), vzl = 0.5 * (v[p - Z] + v[p]);
                    sv[p] = -((uxh * vxh - uxl * vxl) / dx + (fyh * fyh - fyl * fyl) / dy + (wzh * vzh - wzl * vzl) / dz);
                }
                /* w at (i, j, k+1/2) */
                {
                    const double uxh = 0.5 * (u[p] + u[p + Z]), wxh = 0.5 * (w[p] + w[p + X]);
                    const double uxl = 0.5 * (u[p - X] + u[p - X + Z]), wxl = 0.5 * (w[p - X] + w[p]);
                    const double vyh = 0.5 * (v[p] + v[p + Z]), wyh = 0.5 * (w[p] + w[p + Y]);
                    const double vyl = 0.5 * (v[p - Y] + v[p - Y + Z]), wyl = 0.5 * (w[p - Y] + w[p]);
                    const double fzh = 0.5 * (w[p] + w[p + Z]), fzl = 0.5 * (w[p - Z] + w[p]);
                    sw[p] = -((uxh * wxh - uxl * wxl) / dx + (vyh * wyh - vyl * wyl) / dy + (fzh * fzh - fzl * fzl) / dz);
                }
            }
    return ORC_OK;
}

/*
 * Multilinear interpolation over the grid cell of each real position (3
 * slots per point, the first ndim used, each within [0, n - 1] of its axis).
 * For axis j with extent e the cell starts at b = min(floor(x), e - 2)
 * (b = 0 and fraction 0 when e = 1) and the fraction is f = x - b; the lower
 * corner has weight 1 - f, the upper one (b + 1, or b when e = 1) weight f.
 * Corner c of a point takes the upper corner on axis j when bit
 * (ndim - 1 - j) of c is set; its weight is the product over the axes.
 * corners: [n][2^ndim][3] interior coordinates; weights: [n][2^ndim].
 */
int orc_interp(int ndim, const int64_t* shape, int64_t n, const double* pos, int64_t* corners, double* weights) {
    if (ndim < 1 || ndim > 3 || n < 0 || (n > 0 && (!pos || !corners || !weights))) return ORC_EINVAL;
    int nc = 1 << ndim;
    for (int64_t i = 0; i < n; i++) {
        int64_t lo[3], hi[3];
        double frac[3];
        for (int j = 0; j < ndim; j++) {
            double x = pos[3 * i + j];
            int64_t e = shape[j];
            if (!(x >= 0.0 && x <= (double)(e - 1))) return ORC_EINVAL;
            if (e == 1) {
                lo[j] = hi[j] = 0;
                frac[j] = 0.0;
            } else {
                int64_t b = (int64_t)floor(x);
                if (b > e - 2) b = e - 2;
                lo[j] = b;
                hi[j] = b + 1;
                frac[j] = x - (double)b;
            }
        }
        for (int c = 0; c < nc; c++) {
            double w = 1.0;
            int64_t* cp = corners + 3 * (i * nc + c);
            cp[0] = cp[1] = cp[2] = 0;
            for (int j = 0; j < ndim; j++) {
                int up = (c >> (ndim - 1 - j)) & 1;
                cp[j] = up ? hi[j] : lo[j];
                w *= up ? frac[j] : 1.0 - frac[j];
            }
            weights[i * nc + c] = w;
        }
    }
    return ORC_OK;
}

/*
 * The damped leapfrog (see the header): gamma is a full buffer like beta.
 * Sources and receivers as in orc_wave_run; Dirichlet zero halo.
 */
int orc_wave_run_damped(int ndim, const int64_t* shape, int halo, int radius, const double* c,
                        const double* beta, const double* gamma, double* u_n, double* u_nm1, int64_t nsteps,
                        int64_t nsrc, const int64_t* src, const double* src_amp, int64_t nrec, const int64_t* rec,
                        double* traces) {
    og g;
    if (og_init(&g, ndim, shape, halo) || check_common(&g, radius) || nsteps < 0 || !gamma) return ORC_EINVAL;
    if (!pos_list_ok(&g, nsrc, src) || !pos_list_ok(&g, nrec, rec)) return ORC_EINVAL;
    if ((nsrc > 0 && !src_amp) || (nrec > 0 && !traces)) return ORC_EINVAL;
    size_t bytes = sizeof(double) * (size_t)g.total;
    double* a = u_n;
    double* b = u_nm1;
    int64_t lz = og_lo(&g, 0), ly = og_lo(&g, 1), lx = og_lo(&g, 2);
    for (int64_t t = 0; t < nsteps; t++) {
#pragma omp parallel for schedule(static)
        for (int64_t z = lz; z < lz + g.n[0]; z++)
            for (int64_t y = ly; y < ly + g.n[1]; y++)
                for (int64_t x = lx; x < lx + g.n[2]; x++) {
                    int64_t p = z * g.s[0] + y * g.s[1] + x;
                    double lap = star_at(&g, radius, c, a, p);
                    b[p] = (2.0 * a[p] - (1.0 - gamma[p]) * b[p] + beta[p] * lap) / (1.0 + gamma[p]);
                }
        for (int64_t s = 0; s < nsrc; s++) b[og_pos(&g, src + 3 * s)] += src_amp[t * nsrc + s];
        for (int64_t r = 0; r < nrec; r++) traces[t * nrec + r] = b[og_pos(&g, rec + 3 * r)];
        double* tmp = a;
        a = b;
        b = tmp;
    }
    if (a != u_n) {
        double* tmp = (double*)malloc(bytes);
        if (!tmp) return ORC_ENOMEM;
        memcpy(tmp, a, bytes);
        memcpy(u_nm1, u_n, bytes);
        memcpy(u_n, tmp, bytes);
        free(tmp);
    }
    return ORC_OK;
}

int orc_abi_version(void) { return 1; }
