/*
 * Oracle particle step, FP64, plain loops.  TEST INFRASTRUCTURE ONLY: called from the
 * tests, the smoke check and the benchmark's CPU-baseline leg, never from the product.
 *
 * One particle at a time, in the order of the PIC cycle of Sec. II-A:
 *   1. gather E = sum_i e_i W1_i(x) and B = sum_f b_f W2_f(x) at the particle (Sec. II-A);
 *   2. relativistic Boris push of u = gamma v (Sec. III-B names Boris as the comparison
 *      pusher; the relativistic form is Boris 1970): half electric kick, magnetic
 *      rotation, half electric kick; then x^{n+1} = x^n + dt v^{n+1/2};
 *   3. the straight path x^n -> x^{n+1} is followed through the mesh (Alg. 1): in the
 *      current tet, the exit point is where the path meets the plane of a face, i.e. the
 *      first t in [0,1] with lambda_k(x_s + t d) = 0 (eq. (intersection), read as the face
 *      plane; barycentric coordinates are affine so this is a closed form), the path is
 *      cut there, and the walk continues in the neighbouring tet;
 *   4. each piece of path inside one tet adds q w * integral of W1_i . dr to every edge of
 *      that tet (eqs. (gaussredo)-(G): the time integral of the current equals this path
 *      integral).  Along a straight piece W1_ab . dr = lambda_a d lambda_b - lambda_b d
 *      lambda_a is constant, so the one-point (midpoint) rule is exact.
 * A path that reaches a boundary face ends there (absorbing wall, after depositing up to
 * the wall).  Positions are Cartesian; barycentric coordinates are recomputed from them.
 */
#include <math.h>
#include <stdint.h>

#define ORC_C_LIGHT 299792458.0

static const int LOC_E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int LOC_F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

typedef struct {
    int64_t n_tets;
    const double *xyz;        /* [n_nodes][3] */
    const int64_t *tets;      /* [n_tets][4], node ids ascending */
    const int64_t *tet_edges; /* [n_tets][6] */
    const int64_t *tet_faces; /* [n_tets][4], face opposite local vertex k */
    const int64_t *nbr;       /* [n_tets][4], tet across face k, -1 = boundary */
    const double *grad;       /* [n_tets][4][3] grad lambda_k */
} orc_mesh;

typedef struct {
    int64_t n_crossings;
    int64_t max_crossings;
    int64_t n_absorbed;
    int64_t n_cap_exceeded;
} orc_push_stats;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void bary(const orc_mesh *m, int64_t t, const double *x, double lam[4])
{
    for (int k = 0; k < 4; k++) {
        const double *ra = m->xyz + 3 * m->tets[4 * t + LOC_F[k][0]];
        double d[3] = {x[0] - ra[0], x[1] - ra[1], x[2] - ra[2]};
        lam[k] = dot3(d, m->grad + 12 * t + 3 * k);
    }
}

/* E and B at barycentric point lam of tet t (full Whitney-1 and Whitney-2 expansions). */
static void gather(const orc_mesh *m, int64_t t, const double lam[4], const double *e, const double *b,
                   double E[3], double B[3])
{
    const double *g = m->grad + 12 * t;
    E[0] = E[1] = E[2] = 0.0;
    B[0] = B[1] = B[2] = 0.0;
    for (int i = 0; i < 6; i++) {
        int a = LOC_E[i][0], c = LOC_E[i][1];
        double ei = e[m->tet_edges[6 * t + i]];
        for (int d = 0; d < 3; d++)
            E[d] += ei * (lam[a] * g[3 * c + d] - lam[c] * g[3 * a + d]);
    }
    for (int k = 0; k < 4; k++) {
        int i = LOC_F[k][0], j = LOC_F[k][1], l = LOC_F[k][2];
        double cjl[3], cli[3], cij[3];
        cross3(g + 3 * j, g + 3 * l, cjl);
        cross3(g + 3 * l, g + 3 * i, cli);
        cross3(g + 3 * i, g + 3 * j, cij);
        double bf = b[m->tet_faces[4 * t + k]];
        for (int d = 0; d < 3; d++)
            B[d] += bf * 2.0 * (lam[i] * cjl[d] + lam[j] * cli[d] + lam[l] * cij[d]);
    }
}

/* Relativistic Boris: u <- u^{n+1/2} from u^{n-1/2}, fields at x^n. */
void orc_boris(double q, double mass, double dt, const double E[3], const double B[3], double u[3])
{
    const double c2 = ORC_C_LIGHT * ORC_C_LIGHT;
    double h = q * dt / (2.0 * mass);
    double um[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
    double gm = sqrt(1.0 + dot3(um, um) / c2);
    double tv[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
    double tt = dot3(tv, tv);
    double sv[3] = {2.0 * tv[0] / (1.0 + tt), 2.0 * tv[1] / (1.0 + tt), 2.0 * tv[2] / (1.0 + tt)};
    double c1[3], c2v[3];
    cross3(um, tv, c1);
    double up[3] = {um[0] + c1[0], um[1] + c1[1], um[2] + c1[2]};
    cross3(up, sv, c2v);
    for (int d = 0; d < 3; d++)
        u[d] = um[d] + c2v[d] + h * E[d];
}

static void deposit(const orc_mesh *m, int64_t t, const double *xs, const double *xe, double qw, double *dg)
{
    double ls[4], le[4];
    bary(m, t, xs, ls);
    bary(m, t, xe, le);
    for (int i = 0; i < 6; i++) {
        int a = LOC_E[i][0], c = LOC_E[i][1];
        double ma = 0.5 * (ls[a] + le[a]), mc = 0.5 * (ls[c] + le[c]);
        double da = le[a] - ls[a], dc = le[c] - ls[c];
        dg[m->tet_edges[6 * t + i]] += qw * (ma * dc - mc * da);
    }
}

static int entry_vertex(const orc_mesh *m, int64_t from, int64_t to)
{
    for (int k = 0; k < 4; k++) {
        int64_t v = m->tets[4 * to + k];
        int shared = 0;
        for (int j = 0; j < 4; j++)
            shared |= (m->tets[4 * from + j] == v);
        if (!shared)
            return k;
    }
    return -1;
}

/*
 * Follow the straight path x_s -> x_s + d starting in tet t.  Deposits into dg when dg is
 * not NULL; records up to max_rec crossing points/tets when rec_* are not NULL.
 * Returns 0 = ended inside the mesh, 1 = absorbed at the boundary, 2 = crossing cap hit.
 * On return x_s holds the end point and *t the tet holding it.
 */
static int walk(const orc_mesh *m, int64_t *t_io, double x_s[3], const double d_in[3], double qw, double *dg,
                int cap, int64_t *n_cross, int64_t *rec_tets, double *rec_pts, int64_t max_rec)
{
    int64_t t = *t_io;
    double d[3] = {d_in[0], d_in[1], d_in[2]};
    int entry = -1;
    int64_t nc = 0;
    for (;;) {
        double lam[4];
        bary(m, t, x_s, lam);
        const double *g = m->grad + 12 * t;
        double best = INFINITY;
        int kb = -1;
        for (int k = 0; k < 4; k++) {
            if (k == entry)
                continue;
            double s = dot3(g + 3 * k, d);
            if (s < 0.0) {
                double tk = lam[k] / (-s);
                if (tk < best) {
                    best = tk;
                    kb = k;
                }
            }
        }
        double xe[3];
        if (kb < 0 || best >= 1.0) {
            for (int c = 0; c < 3; c++)
                xe[c] = x_s[c] + d[c];
            if (dg)
                deposit(m, t, x_s, xe, qw, dg);
            for (int c = 0; c < 3; c++)
                x_s[c] = xe[c];
            *t_io = t;
            *n_cross = nc;
            return 0;
        }
        for (int c = 0; c < 3; c++)
            xe[c] = x_s[c] + best * d[c];
        if (dg)
            deposit(m, t, x_s, xe, qw, dg);
        for (int c = 0; c < 3; c++)
            x_s[c] = xe[c];
        int64_t nb = m->nbr[4 * t + kb];
        if (rec_tets && nc < max_rec) {
            rec_tets[nc] = nb;
            for (int c = 0; c < 3; c++)
                rec_pts[3 * nc + c] = xe[c];
        }
        if (nb < 0) {
            *t_io = t;
            *n_cross = nc;
            return 1;
        }
        nc++;
        if (nc > cap) {
            *t_io = t;
            *n_cross = nc;
            return 2;
        }
        entry = entry_vertex(m, t, nb);
        for (int c = 0; c < 3; c++)
            d[c] *= (1.0 - best);
        t = nb;
    }
}

/* Barycentric coordinates of points x[n][3] in tets tet[n] -> lam[n][4]. */
void orc_barycentric(const orc_mesh *m, int64_t n, const int64_t *tet, const double *x, double *lam)
{
    for (int64_t p = 0; p < n; p++)
        bary(m, tet[p], x + 3 * p, lam + 4 * p);
}

/* Fields E, B at points x[n] in tets tet[n]. */
void orc_gather(const orc_mesh *m, int64_t n, const int64_t *tet, const double *x, const double *e,
                const double *b, double *E, double *B)
{
    for (int64_t p = 0; p < n; p++) {
        double lam[4];
        bary(m, tet[p], x + 3 * p, lam);
        gather(m, tet[p], lam, e, b, E + 3 * p, B + 3 * p);
    }
}

/* Trace one straight path (no deposit); returns the walk status, fills crossings. */
int orc_trace(const orc_mesh *m, int64_t t0, const double *x0, const double *d, int cap, int64_t *t_end,
              double *x_end, int64_t *n_cross, int64_t *rec_tets, double *rec_pts, int64_t max_rec)
{
    double xs[3] = {x0[0], x0[1], x0[2]};
    int64_t t = t0;
    int st = walk(m, &t, xs, d, 0.0, 0, cap, n_cross, rec_tets, rec_pts, max_rec);
    *t_end = t;
    x_end[0] = xs[0];
    x_end[1] = xs[1];
    x_end[2] = xs[2];
    return st;
}

/* Deposit only: the path x0 -> x0 + d from tet t0, current added to dg. */
int orc_deposit_path(const orc_mesh *m, int64_t t0, const double *x0, const double *d, double qw, double *dg,
                     int cap, int64_t *t_end, double *x_end)
{
    double xs[3] = {x0[0], x0[1], x0[2]};
    int64_t t = t0, nc = 0;
    int st = walk(m, &t, xs, d, qw, dg, cap, &nc, 0, 0, 0);
    *t_end = t;
    x_end[0] = xs[0];
    x_end[1] = xs[1];
    x_end[2] = xs[2];
    return st;
}

/*
 * One particle step for n particles of one species (charge q, mass, macro weight w).
 * x[n][3], u[n][3] (u = gamma v), tet[n], alive[n] are updated in place; the current
 * of every path piece is added to dg (edge vector).  Returns 0, or 2 if any particle hit
 * the crossing cap (that particle is left at the point where it stopped).
 */
int orc_push(const orc_mesh *m, int64_t n, double *x, double *u, int64_t *tet, int8_t *alive, double q,
             double mass, double w, double dt, const double *e, const double *b, double *dg, int cap,
             orc_push_stats *st)
{
    const double c2 = ORC_C_LIGHT * ORC_C_LIGHT;
    int err = 0;
    for (int64_t p = 0; p < n; p++) {
        if (!alive[p])
            continue;
        int64_t t = tet[p];
        double *xp = x + 3 * p, *up = u + 3 * p;
        double lam[4], E[3], B[3];
        bary(m, t, xp, lam);
        gather(m, t, lam, e, b, E, B);
        orc_boris(q, mass, dt, E, B, up);
        double gam = sqrt(1.0 + dot3(up, up) / c2);
        double d[3] = {dt * up[0] / gam, dt * up[1] / gam, dt * up[2] / gam};
        int64_t nc = 0;
        int s = walk(m, &t, xp, d, q * w, dg, cap, &nc, 0, 0, 0);
        tet[p] = t;
        st->n_crossings += nc;
        if (nc > st->max_crossings)
            st->max_crossings = nc;
        if (s == 1) {
            alive[p] = 0;
            st->n_absorbed++;
        } else if (s == 2) {
            st->n_cap_exceeded++;
            err = 2;
        }
    }
    return err;
}
