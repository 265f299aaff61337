/*
 * gribov_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, double-precision CPU reference for the random-start
 * Landau-gauge relaxation of compact U(1) lattice gauge fields (Mehta &
 * Schroeck, "Enumerating Copies in the First Gribov Region on the Lattice in
 * up to four Dimensions").  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the HIP path.
 *
 * What it computes, per start, in the paper's order:
 *   1. lattice, periodic neighbours (Sec. I, compact U(1) paragraph) and a
 *      proper colouring for the checkerboard (Sec. III);
 *   2. U = exp(i phi) (Sec. I, compact U(1) paragraph);
 *   3. random start g_i = exp(i theta_i), theta from Philox4x64-10 (Sec. III);
 *   4. colour-by-colour local maximisation, eqs. (4)-(5), written in the
 *      convention of eq. (3), optionally over-relaxed;
 *   5. stopping test on the lattice divergence (Sec. III; gradient of eq. (3));
 *   6. the functional F of eq. (3) and x = F/(d V) (Sec. III, the map of x
 *      onto an integer grid of resolution 1e-8);
 *   7. an integer key: the wrap numbers of the gauge-transformed link angles
 *      per plaquette and per lattice line (global phase removed, Sec. I).
 * The Faddeev-Popov spectrum and the copy table are formed in oracle.py.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *   - sign convention: eq. (3) is authoritative; the local optimum is
 *     g_i = S_i/|S_i| with S_i = sum_mu [U_{i,mu} g_{i+mu} + conj(U_{i-mu,mu}) g_{i-mu}],
 *     which is the paper's "phase of K_i^*" rule with theta -> -theta;
 *   - over-relaxation (the paper uses none; the workloads ask for omega=1.7):
 *     g <- v/|v| with v = (1 - omega) g + omega S/|S|, the step from g towards
 *     the local optimum S/|S| stretched by omega and put back on the unit
 *     circle (for |g| = 1 this is g w/|w| with w = 1 + omega (conj(g) S/|S| - 1));
 *   - stopping: D = (1/V) sum_i div_i^2 < eps with div_i = Im(conj(g_i) S_i),
 *     evaluated on the post-sweep state, per start (never across starts);
 *     the paper's max |div| < eps rule is available as stop_norm = 1;
 *   - colouring: colour(i) = (sum_mu x_mu) mod K, K = 2 when every extent is
 *     even, else the smallest K >= 3 dividing every extent;
 *   - |S_i| = 0 leaves g_i unchanged.
 *
 * Compiled with -ffp-contract=off so every product and sum rounds as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 4
static const double OR_PI = 3.14159265358979311599796346854;     /* fl(pi) */
static const double OR_TWO_PI = 6.28318530717958623199592693709; /* 2 fl(pi) */

enum { OR_UNSET = 0, OR_CONVERGED = 1, OR_NONCONVERGED = 2, OR_BADNUM = 3 };

/* Per-start result.  Layout mirrored by a numpy structured dtype in oracle.py. */
typedef struct {
    int32_t status;
    int32_t sweeps32;      /* sweeps done in the single-precision phase */
    int32_t sweeps64;      /* sweeps done in double precision */
    int32_t n_elems;       /* key payload length */
    double F;              /* eq. (3) at the final state */
    double x;              /* F / (d V) */
    double D;              /* final stopping norm */
    double cut_margin;     /* min over links of pi - |a_l| */
    uint64_t key_hi;
    uint64_t key_lo;
    uint32_t paper_X;      /* trunc(x * 1e8) */
    int32_t key_overflow;  /* payload entry outside int8 */
} or_record;

/* ------------------------------------------------------------------ */
/* Lattice geometry: periodic boundary conditions (Sec. I).            */
/* Site index i = sum_mu x_mu s_mu, s_0 = 1, s_mu = s_{mu-1} N_{mu-1}. */
/* ------------------------------------------------------------------ */
typedef struct {
    int d;
    int n[OR_MAXD];
    int64_t s[OR_MAXD];
    int64_t V;
    int K;            /* number of colours */
    int32_t *fwd;     /* [d][V] */
    int32_t *bwd;     /* [d][V] */
    int32_t *colour;  /* [V] */
} or_lattice;

static int or_num_colours(int d, const int *n)
{
    int all_even = 1;
    for (int mu = 0; mu < d; ++mu)
        if (n[mu] % 2) all_even = 0;
    if (all_even) return 2;
    int nmin = n[0];
    for (int mu = 1; mu < d; ++mu)
        if (n[mu] < nmin) nmin = n[mu];
    for (int K = 3; K <= nmin; ++K) {
        int ok = 1;
        for (int mu = 0; mu < d; ++mu)
            if (n[mu] % K) ok = 0;
        if (ok) return K;
    }
    return 0;
}

static void or_coords(const or_lattice *L, int64_t i, int *x)
{
    for (int mu = 0; mu < L->d; ++mu) {
        x[mu] = (int)(i % L->n[mu]);
        i /= L->n[mu];
    }
}

static int or_lattice_init(or_lattice *L, int d, const int *n)
{
    if (d < 1 || d > OR_MAXD) return -1;
    L->d = d;
    L->V = 1;
    for (int mu = 0; mu < d; ++mu) {
        if (n[mu] < 2) return -1;
        L->n[mu] = n[mu];
        L->s[mu] = L->V;
        L->V *= n[mu];
    }
    L->K = or_num_colours(d, n);
    L->fwd = (int32_t *)malloc(sizeof(int32_t) * d * L->V);
    L->bwd = (int32_t *)malloc(sizeof(int32_t) * d * L->V);
    L->colour = (int32_t *)malloc(sizeof(int32_t) * L->V);
    int x[OR_MAXD];
    for (int64_t i = 0; i < L->V; ++i) {
        or_coords(L, i, x);
        int sum = 0;
        for (int mu = 0; mu < d; ++mu) {
            sum += x[mu];
            int xf = (x[mu] + 1) % n[mu];
            int xb = (x[mu] + n[mu] - 1) % n[mu];
            L->fwd[mu * L->V + i] = (int32_t)(i + (int64_t)(xf - x[mu]) * L->s[mu]);
            L->bwd[mu * L->V + i] = (int32_t)(i + (int64_t)(xb - x[mu]) * L->s[mu]);
        }
        L->colour[i] = L->K ? sum % L->K : 0;
    }
    return L->K ? 0 : -2;
}

static void or_lattice_free(or_lattice *L)
{
    free(L->fwd);
    free(L->bwd);
    free(L->colour);
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the */
/* published round function: two 64x64->128 multiplies per round, the  */
/* key bumped by the Weyl constants after every round.                 */
/* ------------------------------------------------------------------ */
static void or_mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        or_mul128(M0, c0, &hi0, &lo0);
        or_mul128(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = (r >> 11) 2^-53 in [0,1); angle = fl(fl(u * 2pi) - pi) in [-pi, pi). */
static double or_angle(uint64_t r)
{
    double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);
    double t = u * OR_TWO_PI;
    return t - OR_PI;
}

/* Random start (Sec. III: one Philox-initialised gauge transformation per
 * sample).  Site i draws counter (i/4, start_id, orbit_index, 0x53) under key
 * (start_seed, 1) and takes word i%4. */
void oracle_start_angles(uint64_t start_seed, uint64_t start_id, uint64_t orbit_index,
                         int64_t V, double *theta)
{
    uint64_t key[2] = {start_seed, 1};
    for (int64_t b = 0; b * 4 < V; ++b) {
        uint64_t ctr[4] = {(uint64_t)b, start_id, orbit_index, 0x53};
        uint64_t out[4];
        oracle_philox4x64_10(ctr, key, out);
        for (int k = 0; k < 4 && b * 4 + k < V; ++k) theta[b * 4 + k] = or_angle(out[k]);
    }
}

/* SplitMix64 output function (Steele, Lea, Flood 2014). */
uint64_t oracle_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ */
/* Local update, eqs. (4)-(5) in the eq. (3) convention.               */
/* ------------------------------------------------------------------ */

/* S_i = sum_mu [U_{i,mu} g_{i+mu} + conj(U_{i-mu,mu}) g_{i-mu}], mu ascending,
 * forward term before backward term. */
static void or_staple64(const or_lattice *L, const double *Ur, const double *Ui,
                        const double *gr, const double *gi, int64_t i,
                        double *sr, double *si)
{
    double ar = 0.0, ai = 0.0;
    for (int mu = 0; mu < L->d; ++mu) {
        int64_t f = L->fwd[mu * L->V + i];
        int64_t b = L->bwd[mu * L->V + i];
        double ur = Ur[mu * L->V + i], ui = Ui[mu * L->V + i];
        ar = ar + (ur * gr[f] - ui * gi[f]);
        ai = ai + (ur * gi[f] + ui * gr[f]);
        double vr = Ur[mu * L->V + b], vi = -Ui[mu * L->V + b];
        ar = ar + (vr * gr[b] - vi * gi[b]);
        ai = ai + (vr * gi[b] + vi * gr[b]);
    }
    *sr = ar;
    *si = ai;
}

static void or_staple32(const or_lattice *L, const float *Ur, const float *Ui,
                        const float *gr, const float *gi, int64_t i,
                        float *sr, float *si)
{
    float ar = 0.0f, ai = 0.0f;
    for (int mu = 0; mu < L->d; ++mu) {
        int64_t f = L->fwd[mu * L->V + i];
        int64_t b = L->bwd[mu * L->V + i];
        float ur = Ur[mu * L->V + i], ui = Ui[mu * L->V + i];
        ar = ar + (ur * gr[f] - ui * gi[f]);
        ai = ai + (ur * gi[f] + ui * gr[f]);
        float vr = Ur[mu * L->V + b], vi = -Ui[mu * L->V + b];
        ar = ar + (vr * gr[b] - vi * gi[b]);
        ai = ai + (vr * gi[b] + vi * gr[b]);
    }
    *sr = ar;
    *si = ai;
}

/* One full sweep: colours 0..K-1 in order; inside a colour the sites are
 * independent (Sec. III, checkerboard), taken here in ascending order. */
static void or_sweep64(const or_lattice *L, const double *Ur, const double *Ui,
                       double *gr, double *gi, double omega)
{
    for (int c = 0; c < L->K; ++c) {
        for (int64_t i = 0; i < L->V; ++i) {
            if (L->colour[i] != c) continue;
            double sr, si;
            or_staple64(L, Ur, Ui, gr, gi, i, &sr, &si);
            double n2 = sr * sr + si * si;
            if (n2 == 0.0) continue;
            double nrm = sqrt(n2);
            double hr = sr / nrm, hi = si / nrm;
            if (omega == 1.0) {
                gr[i] = hr;
                gi[i] = hi;
            } else {
                double vr = (1.0 - omega) * gr[i] + omega * hr;
                double vi = (1.0 - omega) * gi[i] + omega * hi;
                double vn = sqrt(vr * vr + vi * vi);
                gr[i] = vr / vn;
                gi[i] = vi / vn;
            }
        }
    }
}

static void or_sweep32(const or_lattice *L, const float *Ur, const float *Ui,
                       float *gr, float *gi, float omega)
{
    for (int c = 0; c < L->K; ++c) {
        for (int64_t i = 0; i < L->V; ++i) {
            if (L->colour[i] != c) continue;
            float sr, si;
            or_staple32(L, Ur, Ui, gr, gi, i, &sr, &si);
            float n2 = sr * sr + si * si;
            if (n2 == 0.0f) continue;
            float nrm = sqrtf(n2);
            float hr = sr / nrm, hi = si / nrm;
            if (omega == 1.0f) {
                gr[i] = hr;
                gi[i] = hi;
            } else {
                float vr = (1.0f - omega) * gr[i] + omega * hr;
                float vi = (1.0f - omega) * gi[i] + omega * hi;
                float vn = sqrtf(vr * vr + vi * vi);
                gr[i] = vr / vn;
                gi[i] = vi / vn;
            }
        }
    }
}

/* Stopping norm on the current state.  div_i = Im(conj(g_i) S_i) = -dF/dtheta_i.
 * stop_norm 0: (1/V) sum_i div_i^2.  stop_norm 1: max_i |div_i| (the paper's rule). */
static double or_norm64(const or_lattice *L, const double *Ur, const double *Ui,
                        const double *gr, const double *gi, int stop_norm)
{
    double acc = 0.0;
    for (int64_t i = 0; i < L->V; ++i) {
        double sr, si;
        or_staple64(L, Ur, Ui, gr, gi, i, &sr, &si);
        double dv = gr[i] * si - gi[i] * sr;
        if (stop_norm == 1) {
            if (fabs(dv) > acc) acc = fabs(dv);
        } else {
            acc = acc + dv * dv;
        }
    }
    return stop_norm == 1 ? acc : acc / (double)L->V;
}

/* Single-precision phase: div_i in float, squares summed in double. */
static double or_norm32(const or_lattice *L, const float *Ur, const float *Ui,
                        const float *gr, const float *gi, int stop_norm)
{
    double acc = 0.0;
    for (int64_t i = 0; i < L->V; ++i) {
        float sr, si;
        or_staple32(L, Ur, Ui, gr, gi, i, &sr, &si);
        float dv = gr[i] * si - gi[i] * sr;
        double d = (double)dv;
        if (stop_norm == 1) {
            if (fabs(d) > acc) acc = fabs(d);
        } else {
            acc = acc + d * d;
        }
    }
    return stop_norm == 1 ? acc : acc / (double)L->V;
}

/* ------------------------------------------------------------------ */
/* Observables and key (eq. (3); global phase removal, Sec. I).        */
/* ------------------------------------------------------------------ */

/* u_l = conj(g_i) U_{i,mu} g_{i+mu}; a_l = arg u_l in (-pi, pi];
 * F = sum_l (1 - Re u_l). */
static double or_links(const or_lattice *L, const double *Ur, const double *Ui,
                       const double *gr, const double *gi, double *a, double *w,
                       double *cut_margin)
{
    double F = 0.0;
    double margin = OR_PI;
    for (int mu = 0; mu < L->d; ++mu) {
        for (int64_t i = 0; i < L->V; ++i) {
            int64_t l = mu * L->V + i;
            int64_t f = L->fwd[l];
            double tr = Ur[l] * gr[f] - Ui[l] * gi[f];
            double ti = Ur[l] * gi[f] + Ui[l] * gr[f];
            double ur = gr[i] * tr + gi[i] * ti;
            double ui = gr[i] * ti - gi[i] * tr;
            F = F + (1.0 - ur);
            if (w) w[l] = ur;
            double al = atan2(ui, ur);
            a[l] = al;
            double m = OR_PI - fabs(al);
            if (m < margin) margin = m;
        }
    }
    if (cut_margin) *cut_margin = margin;
    return F;
}

static int64_t or_n_plaquettes(const or_lattice *L) { return (int64_t)L->d * (L->d - 1) / 2 * L->V; }

static int64_t or_n_lines(const or_lattice *L)
{
    int64_t n = 0;
    for (int mu = 0; mu < L->d; ++mu) n += L->V / L->n[mu];
    return n;
}

int64_t oracle_key_length(int d, const int *n)
{
    or_lattice L;
    int rc = or_lattice_init(&L, d, n);
    if (rc == -1) return -1;
    int64_t m = or_n_plaquettes(&L) + or_n_lines(&L);
    or_lattice_free(&L);
    return m;
}

/* Integer payload: plaquette wrap numbers n_p for every (mu<nu) in
 * lexicographic order, site ascending, then line windings w_l for every
 * direction mu, lines ordered by the index of their x_mu = 0 site. */
static int or_payload(const or_lattice *L, const double *phi, const double *a, int32_t *e)
{
    int64_t k = 0;
    for (int mu = 0; mu < L->d; ++mu) {
        for (int nu = mu + 1; nu < L->d; ++nu) {
            for (int64_t i = 0; i < L->V; ++i) {
                int64_t fm = L->fwd[mu * L->V + i];
                int64_t fn = L->fwd[nu * L->V + i];
                double A = a[mu * L->V + i] + a[nu * L->V + fm] - a[mu * L->V + fn] - a[nu * L->V + i];
                double P = phi[mu * L->V + i] + phi[nu * L->V + fm] - phi[mu * L->V + fn] - phi[nu * L->V + i];
                e[k++] = (int32_t)rint((A - P) / OR_TWO_PI);
            }
        }
    }
    int x[OR_MAXD];
    for (int mu = 0; mu < L->d; ++mu) {
        for (int64_t i0 = 0; i0 < L->V; ++i0) {
            or_coords(L, i0, x);
            if (x[mu] != 0) continue;
            double sa = 0.0, sp = 0.0;
            int64_t i = i0;
            for (int t = 0; t < L->n[mu]; ++t) {
                sa = sa + a[mu * L->V + i];
                sp = sp + phi[mu * L->V + i];
                i = L->fwd[mu * L->V + i];
            }
            e[k++] = (int32_t)rint((sa - sp) / OR_TWO_PI);
        }
    }
    int overflow = 0;
    for (int64_t j = 0; j < k; ++j)
        if (e[j] < -128 || e[j] > 127) overflow = 1;
    return overflow;
}

/* 128-bit key: lane j sums mix64(c_j ^ (k << 8 | (uint8)e_k)) over payload
 * positions k (mod 2^64), then finalises with mix64(sum + length).  A zero
 * word is mapped to 1 (zero marks an empty table slot in the high word and a
 * slot whose low word is not yet written in the low word). */
static void or_hash(const int32_t *e, int64_t m, uint64_t *hi, uint64_t *lo)
{
    const uint64_t c0 = 0x243F6A8885A308D3ULL, c1 = 0x13198A2E03707344ULL;
    uint64_t h0 = 0, h1 = 0;
    for (int64_t k = 0; k < m; ++k) {
        uint64_t word = ((uint64_t)k << 8) | (uint64_t)(uint8_t)(int8_t)e[k];
        h0 += oracle_mix64(c0 ^ word);
        h1 += oracle_mix64(c1 ^ word);
    }
    h0 = oracle_mix64(h0 + (uint64_t)m);
    h1 = oracle_mix64(h1 + (uint64_t)m);
    if (h0 == 0) h0 = 1;
    if (h1 == 0) h1 = 1;
    *hi = h0;
    *lo = h1;
}

/* ------------------------------------------------------------------ */
/* Per-start solve.                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    double omega;
    double eps32, eps64;
    int32_t precision;    /* 0: double throughout, 1: float sweeps then double polish */
    int32_t stop_norm;    /* 0: mean square, 1: max abs */
    int32_t check_every;
    int32_t fixed;          /* 1: run exactly max_sweeps double sweeps, norm after the last (batch-synchronous pass) */
    int64_t max_sweeps;
    uint64_t start_seed;
    uint64_t orbit_index;
} or_params;

static void or_solve_one(const or_lattice *L, const double *phi, const double *Ur, const double *Ui,
                         const float *Ur32, const float *Ui32, const or_params *p,
                         uint64_t start_id, const double *theta0, or_record *rec,
                         double *g_out, int32_t *payload_out, double *work)
{
    int64_t V = L->V;
    double *theta = work;
    double *gr = theta + V;
    double *gi = gr + V;
    double *a = gi + V;                 /* d V */
    float *gr32 = (float *)(a + L->d * V);
    float *gi32 = gr32 + V;
    int32_t *e = (int32_t *)(gi32 + V);

    memset(rec, 0, sizeof(*rec));
    if (theta0)
        memcpy(theta, theta0, sizeof(double) * V);
    else
        oracle_start_angles(p->start_seed, start_id, p->orbit_index, V, theta);
    for (int64_t i = 0; i < V; ++i) {
        gr[i] = cos(theta[i]);
        gi[i] = sin(theta[i]);
    }
    int check = p->check_every > 0 ? p->check_every : 1;
    int status = OR_NONCONVERGED;
    double D = INFINITY;

    if (p->precision == 1) {
        /* Single-precision bulk: start from the rounded double start. */
        for (int64_t i = 0; i < V; ++i) {
            gr32[i] = (float)gr[i];
            gi32[i] = (float)gi[i];
        }
        int64_t t = 0;
        int done = 0;
        while (t < p->max_sweeps) {
            or_sweep32(L, Ur32, Ui32, gr32, gi32, (float)p->omega);
            ++t;
            if (t % check == 0 || t == p->max_sweeps) {
                D = or_norm32(L, Ur32, Ui32, gr32, gi32, p->stop_norm);
                if (!(D == D)) break;
                if (D < p->eps32) { done = 1; break; }
            }
        }
        rec->sweeps32 = (int32_t)t;
        if (!done) {
            rec->status = (D == D) ? OR_NONCONVERGED : OR_BADNUM;
            rec->D = D;
            return;
        }
        /* Promotion: g64 = normalise((double) g32). */
        for (int64_t i = 0; i < V; ++i) {
            double xr = (double)gr32[i], xi = (double)gi32[i];
            double nn = sqrt(xr * xr + xi * xi);
            gr[i] = xr / nn;
            gi[i] = xi / nn;
        }
    }
    {
        /* The paper stops all concurrently relaxed samples together (Sec. III,
         * stopping criterion); in the fixed mode a sample runs the number of
         * sweeps its batch needed and its norm is tested after the last. */
        int64_t t = 0;
        while (t < p->max_sweeps) {
            or_sweep64(L, Ur, Ui, gr, gi, p->omega);
            ++t;
            if ((!p->fixed && t % check == 0) || t == p->max_sweeps) {
                D = or_norm64(L, Ur, Ui, gr, gi, p->stop_norm);
                if (!(D == D)) { status = OR_BADNUM; break; }
                if (D < p->eps64) {
                    status = OR_CONVERGED;
                    if (!p->fixed) break;
                }
            }
        }
        rec->sweeps64 = (int32_t)t;
    }
    rec->status = status;
    rec->D = D;
    if (g_out) {
        for (int64_t i = 0; i < V; ++i) {
            g_out[2 * i] = gr[i];
            g_out[2 * i + 1] = gi[i];
        }
    }
    if (status != OR_CONVERGED) return;
    double margin;
    double F = or_links(L, Ur, Ui, gr, gi, a, NULL, &margin);
    rec->F = F;
    rec->x = F / ((double)L->d * (double)V);
    rec->cut_margin = margin;
    rec->paper_X = (uint32_t)(rec->x * 1e8);
    int64_t m = or_n_plaquettes(L) + or_n_lines(L);
    rec->n_elems = (int32_t)m;
    rec->key_overflow = or_payload(L, phi, a, e);
    or_hash(e, m, &rec->key_hi, &rec->key_lo);
    if (payload_out) memcpy(payload_out, e, sizeof(int32_t) * m);
}

/* Solve the listed starts.  theta_init: NULL (Philox starts) or [n][V].
 * g_out: NULL or [n][V][2] final state.  payload_out: NULL or [n][m]. */
int oracle_solve(int d, const int *extent, const double *phi,
                 const uint64_t *start_ids, int64_t n_starts, const or_params *p,
                 const double *theta_init, int n_threads,
                 or_record *out, double *g_out, int32_t *payload_out)
{
    or_lattice L;
    int rc = or_lattice_init(&L, d, extent);
    if (rc == -1) return rc;
    if (rc == -2) { or_lattice_free(&L); return rc; }
    int64_t V = L.V;
    int64_t m = or_n_plaquettes(&L) + or_n_lines(&L);
    double *Ur = (double *)malloc(sizeof(double) * d * V);
    double *Ui = (double *)malloc(sizeof(double) * d * V);
    float *Ur32 = (float *)malloc(sizeof(float) * d * V);
    float *Ui32 = (float *)malloc(sizeof(float) * d * V);
    /* U = exp(i phi) (Sec. I). */
    for (int64_t l = 0; l < d * V; ++l) {
        Ur[l] = cos(phi[l]);
        Ui[l] = sin(phi[l]);
        Ur32[l] = (float)Ur[l];
        Ui32[l] = (float)Ui[l];
    }
    size_t work_bytes = sizeof(double) * (3 * V + d * V) + sizeof(float) * 2 * V + sizeof(int32_t) * m + 64;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
    {
        double *work = (double *)malloc(work_bytes);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < n_starts; ++s) {
            or_solve_one(&L, phi, Ur, Ui, Ur32, Ui32, p, start_ids[s],
                         theta_init ? theta_init + s * V : NULL, &out[s],
                         g_out ? g_out + s * 2 * V : NULL,
                         payload_out ? payload_out + s * m : NULL, work);
        }
        free(work);
    }
    free(Ur); free(Ui); free(Ur32); free(Ui32);
    or_lattice_free(&L);
    return 0;
}

/* Observables and key of an arbitrary state g = exp(i theta) (no relaxation).
 * a_out [d][V] link angles, w_out [d][V] link weights Re u_l (both optional). */
int oracle_observe(int d, const int *extent, const double *phi, const double *theta,
                   or_record *rec, int32_t *payload_out, double *a_out, double *w_out)
{
    or_lattice L;
    int rc = or_lattice_init(&L, d, extent);
    if (rc == -1) return rc;
    int64_t V = L.V;
    int64_t m = or_n_plaquettes(&L) + or_n_lines(&L);
    double *Ur = (double *)malloc(sizeof(double) * d * V);
    double *Ui = (double *)malloc(sizeof(double) * d * V);
    double *gr = (double *)malloc(sizeof(double) * V);
    double *gi = (double *)malloc(sizeof(double) * V);
    double *a = (double *)malloc(sizeof(double) * d * V);
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (m + 1));
    for (int64_t l = 0; l < d * V; ++l) { Ur[l] = cos(phi[l]); Ui[l] = sin(phi[l]); }
    for (int64_t i = 0; i < V; ++i) { gr[i] = cos(theta[i]); gi[i] = sin(theta[i]); }
    memset(rec, 0, sizeof(*rec));
    double margin;
    rec->F = or_links(&L, Ur, Ui, gr, gi, a, w_out, &margin);
    rec->x = rec->F / ((double)d * (double)V);
    rec->cut_margin = margin;
    rec->paper_X = (uint32_t)(rec->x * 1e8);
    rec->D = or_norm64(&L, Ur, Ui, gr, gi, 0);
    rec->n_elems = (int32_t)m;
    rec->key_overflow = or_payload(&L, phi, a, e);
    or_hash(e, m, &rec->key_hi, &rec->key_lo);
    rec->status = OR_CONVERGED;
    if (payload_out) memcpy(payload_out, e, sizeof(int32_t) * m);
    if (a_out) memcpy(a_out, a, sizeof(double) * d * V);
    free(Ur); free(Ui); free(gr); free(gi); free(a); free(e);
    or_lattice_free(&L);
    return 0;
}

/* Colouring used by the checkerboard; returns K (0 if none exists). */
int oracle_colouring(int d, const int *extent, int32_t *colour_out)
{
    or_lattice L;
    int rc = or_lattice_init(&L, d, extent);
    if (rc == -1) return -1;
    if (colour_out) memcpy(colour_out, L.colour, sizeof(int32_t) * L.V);
    int K = L.K;
    or_lattice_free(&L);
    return K;
}

/* Neighbour tables (for the tests' independent formulas). */
int oracle_neighbours(int d, const int *extent, int32_t *fwd, int32_t *bwd)
{
    or_lattice L;
    int rc = or_lattice_init(&L, d, extent);
    if (rc == -1) return -1;
    memcpy(fwd, L.fwd, sizeof(int32_t) * d * L.V);
    memcpy(bwd, L.bwd, sizeof(int32_t) * d * L.V);
    or_lattice_free(&L);
    return 0;
}

int oracle_record_size(void) { return (int)sizeof(or_record); }
int oracle_params_size(void) { return (int)sizeof(or_params); }
