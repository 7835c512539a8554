/*
 * gsbs_oracle.c -- plain FP64 CPU oracle of the step-by-step (SBS) Brownian
 * diffusion-reaction of water-radiolysis species in a periodic cube.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The HIP engine never
 * links, loads or calls it, and the two share no source, header, table or
 * constant: everything below is written out again from the paper.
 *
 * Paper: Molina-Hernandez, Goncalves, Chi, Seco, "Advancements in Monte Carlo
 * simulations with gMicroMC: reactive species build-up promotes radical-radical
 * reactions at Flash dose rates" (arXiv 2509.03313).  What each part follows:
 *   - Sec. "Theory of periodic boundary conditions", Eq. (1): PBC 1, a molecule
 *     leaving the cube re-enters on the opposite face after each jump.
 *   - same section, Eq. (2): PBC 2, minimum-image pair separation; the
 *     minimum-image convention needs 2R < L.
 *   - Table 1: the nine reactions R1-R9 and their rate constants; for the
 *     self-recombinations R1, R6, R8 the printed number is 2k and is the input
 *     of the radius computation (Sec. "Physico-chemistry and chemistry updates").
 *   - Table S2: diffusion coefficients (the species table is an input here).
 *   - Supplement, reaction-radius derivation: the time-dependent rate
 *     k_diff(t) = 4 pi R D_AB (1 + R / sqrt(pi D_AB t)) N_A; its steady-state
 *     limit solved for R gives the reaction radius.
 *   - Sec. "Verification of periodic boundary conditions ...": a reaction
 *     happens when two reactants come within R.  For a finite step the oracle
 *     uses the exact probability that the relative coordinate touched R during
 *     the step given its end points (method of images applied to the pair
 *     density p(r,t) of the supplement, with the sign of its erfc argument read
 *     as +(r-R)).
 *
 *   - Sec. "Setup for verification of periodic boundary conditions" and the
 *     discussion of its figure: the stochastic (Gillespie) reference for
 *     homogeneous mixtures, orc_ssa (direct method).
 *   - Extensions of Table 1 (the discussion asks for pH and oxygen
 *     chemistry): zero-order sources in orc_ssa and first-order channels in
 *     orc_step and orc_ssa.
 *
 * Everything is FP64, except the two functions whose names end in _f32: they
 * emulate the single-precision cell binning and candidate test bit for bit so
 * that integer decisions taken in FP32 can be compared exactly.
 *
 * Readings where the paper is silent (product placement, uids, partner
 * matching, the step schedule) are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_SPECIES 16
#define ORC_MAX_REACT 32

/* Chemistry: species diffusion coefficients (nm^2/ns) and reactions
 * (rate constant in 1e10 L/mol/s, as printed in Table 1). */
typedef struct {
    int32_t ns;
    int32_t nr;
    double D[ORC_MAX_SPECIES];
    int32_t ra[ORC_MAX_REACT];
    int32_t rb[ORC_MAX_REACT];
    double k_in[ORC_MAX_REACT];
    int32_t nprod[ORC_MAX_REACT];
    int32_t prod[ORC_MAX_REACT][3];
    int32_t keep_b[ORC_MAX_REACT]; /* test-only sink: reactant of species rb survives untouched */
    double c_cut;                  /* candidate cutoff r_c = R + c_cut * sqrt(2 D_AB dt) */
    int32_t rounds;                /* rounds of mutual-best matching per step */
    int32_t contact_only;          /* 1: react only if the pair is within R at the start or end */
    int32_t brute;                 /* 1: all-pairs candidate search instead of the cell list */
    /* First-order (pseudo-first-order scavenging) channels, an extension: a
     * molecule of species s turns into fo_prod[s][0] (plus fo_prod[s][1]
     * when fo_nprod[s] == 2; removed when 0) at rate fo_k[s] per ns. */
    double fo_k[ORC_MAX_SPECIES];
    int32_t fo_nprod[ORC_MAX_SPECIES];
    int32_t fo_prod[ORC_MAX_SPECIES][2];
} orc_chem;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128 multiplies, the     */
/* Weyl key schedule between rounds.                                         */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 24 bits of a word, (k + 1/2) 2^-24: exact in FP64. */
double orc_u24(uint64_t w)
{
    return ((double)(w >> 40) + 0.5) * (1.0 / 16777216.0);
}

/* Box-Muller: three standard normals from one Philox block. */
void orc_gauss3(const uint64_t w[4], double z[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = orc_u24(w[0]), u1 = orc_u24(w[1]);
    double u2 = orc_u24(w[2]), u3 = orc_u24(w[3]);
    double ra = sqrt(-2.0 * log(u0));
    double rb = sqrt(-2.0 * log(u2));
    z[0] = ra * cos(two_pi * u1);
    z[1] = ra * sin(two_pi * u1);
    z[2] = rb * cos(two_pi * u3);
}

/* PBC 1, Eq. (1).  A Gaussian jump can exceed one box edge, so the shift is a
 * whole number of edges; the two clamps are Eq. (1) itself. */
double orc_wrap(double x, double L)
{
    x -= L * floor((x + 0.5 * L) / L);
    if (x >= 0.5 * L) x -= L;
    if (x < -0.5 * L) x += L;
    return x;
}

/* PBC 2, Eq. (2): minimum image of a separation between wrapped positions. */
double orc_minimg(double d, double L)
{
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

/* Reaction radius (nm) from the Table 1 rate constant k_in (1e10 L/mol/s) and
 * D_AB = D_A + D_B (nm^2/ns): steady-state limit of the supplement's k_diff(t)
 * equation, k = 4 pi R D_AB N_A.  For R1/R6/R8 k_in is the printed 2k, which is
 * the supplement's 2 k_diff equation. 1e10 L/mol/s = 1e25/N_A nm^3/ns. */
double orc_radius(double k_in, double Dab)
{
    const double NA = 6.02214076e23;
    const double pi = 3.14159265358979323846264338327950;
    double k_nm3_per_ns = k_in * (1e25 / NA);
    return k_nm3_per_ns / (4.0 * pi * Dab);
}

/* Candidate cutoff: R plus c standard deviations of the relative jump. */
double orc_cutoff(double R, double Dab, double dt, double c)
{
    return R + c * sqrt(2.0 * Dab * dt);
}

/* Probability that a pair whose separation was r0 at the start of a step and
 * r1 at its end came within R during the step, s = D_AB * dt.
 * The free radial propagator of u = r p is a Gaussian minus its image at -r0;
 * with an absorbing sphere the image sits at 2R - r0 (supplement, the
 * boundary conditions of p(r,t)).  The ratio of the two propagators is the
 * survival probability given the end points, so
 *   P = [exp(-(r0-R)(r1-R)/s) - exp(-r0 r1/s)] / [1 - exp(-r0 r1/s)],
 * written with expm1 to stay accurate when s is large.  Pairs already within
 * R react with certainty (a reaction happens inside R). */
double orc_bridge(double r0, double r1, double R, double s)
{
    if (r0 <= R || r1 <= R) return 1.0;
    if (s <= 0.0) return 0.0;
    double a = (r0 - R) * (r1 - R) / s;
    double b = R * (r0 + r1 - R) / s;
    double c = r0 * r1 / s;
    return exp(-a) * expm1(-b) / expm1(-c);
}

/* Largest step for which every reaction's cutoff stays below L/2, so that the
 * minimum image of Eq. (2) is unique for every candidate (the paper's 2R < L,
 * strengthened to the cutoff). */
double orc_dt_max(const orc_chem* c, double L)
{
    double best = INFINITY;
    for (int r = 0; r < c->nr; ++r) {
        double Dab = c->D[c->ra[r]] + c->D[c->rb[r]];
        if (Dab <= 0.0) continue;
        double R = orc_radius(c->k_in[r], Dab);
        double room = (0.5 * L - R) / c->c_cut;
        if (room <= 0.0) return 0.0;
        double dt = room * room / (2.0 * Dab);
        if (dt < best) best = dt;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Step schedule.  Reading of the paper (it gives none): after each injection */
/* time tau the step end times are tau + dt0 * ratio^j, j = 0,1,...  (times  */
/* log-spaced from tau + dt0), until the next injection; every record time,  */
/* injection time and the target time is a step end; a lattice point closer  */
/* than 1e-9 (relative) to one of those is dropped; gaps above dt_max are cut */
/* into equal sub-steps.                                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double t; int ev; } orc_tp;

static int orc_tp_cmp(const void* a, const void* b)
{
    const orc_tp* x = (const orc_tp*)a;
    const orc_tp* y = (const orc_tp*)b;
    if (x->t < y->t) return -1;
    if (x->t > y->t) return 1;
    return y->ev - x->ev; /* events before lattice points at equal times */
}

int64_t orc_schedule(double t_start, double t_end, int32_t n_anchor, const double* anchors,
                     int32_t n_ev, const double* events, double dt0, double ratio, double dt_max,
                     double* out, int64_t max_out)
{
    int64_t cap = 1024, n = 0;
    orc_tp* pts = (orc_tp*)malloc(sizeof(orc_tp) * cap);
    for (int32_t k = 0; k < n_anchor; ++k) {
        double a = anchors[k];
        double next = (k + 1 < n_anchor) ? anchors[k + 1] : INFINITY;
        for (int64_t j = 0;; ++j) {
            double p = a + dt0 * pow(ratio, (double)j);
            if (p >= next || p > t_end) break;
            if (p <= t_start) continue;
            if (n == cap) { cap *= 2; pts = (orc_tp*)realloc(pts, sizeof(orc_tp) * cap); }
            pts[n].t = p; pts[n].ev = 0; ++n;
        }
    }
    for (int32_t k = 0; k <= n_ev; ++k) {
        double e = (k < n_ev) ? events[k] : t_end;
        if (!(e > t_start) || e > t_end) continue;
        if (n == cap) { cap *= 2; pts = (orc_tp*)realloc(pts, sizeof(orc_tp) * cap); }
        pts[n].t = e; pts[n].ev = 1; ++n;
    }
    qsort(pts, (size_t)n, sizeof(orc_tp), orc_tp_cmp);
    /* merge near-coincident points, events win */
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        orc_tp q = pts[i];
        double prev = (m > 0) ? pts[m - 1].t : t_start;
        int prev_ev = (m > 0) ? pts[m - 1].ev : 1;
        if (q.t - prev <= 1e-9 * fabs(q.t)) {
            if (m > 0 && q.ev && !prev_ev) { pts[m - 1] = q; continue; }
            if (!q.ev) continue;
            if (q.t == prev) continue;
        }
        pts[m++] = q;
    }
    /* cap the step */
    int64_t nout = 0;
    double prev = t_start;
    for (int64_t i = 0; i < m; ++i) {
        double g = pts[i].t - prev;
        if (g > dt_max) {
            int64_t ns = (int64_t)ceil(g / dt_max);
            for (int64_t s = 1; s < ns; ++s) {
                if (out && nout < max_out) out[nout] = prev + g * (double)s / (double)ns;
                ++nout;
            }
        }
        if (out && nout < max_out) out[nout] = pts[i].t;
        ++nout;
        prev = pts[i].t;
    }
    free(pts);
    return nout;
}

/* ------------------------------------------------------------------------ */
/* One periodic box (one instance).                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double L;
    uint64_t key[2];      /* Philox key = (seed, instance id) */
    int64_t n, cap;
    double* x;            /* end-of-step positions, 3 per molecule */
    double* x0;           /* start-of-step positions */
    int32_t* sp;
    uint64_t* uid;
    uint64_t next_uid;
    int64_t step;
    double t;
    double edep_eV;
    /* diagnostics of the last step */
    int64_t n_cand, n_acc, n_react;
    /* optional log of the last step's pairs (uids, probability, uniform) */
    int32_t log_mode;     /* 0 none, 1 accepted pairs, 2 every candidate */
    int64_t log_n, log_cap;
    uint64_t* log_uid;    /* 2 per pair: lower uid, higher uid */
    double* log_P;
    uint32_t* log_u24;
    int32_t* log_flag;    /* bit0 accepted, bit1 reacted */
    int32_t* log_rx;
} orc_inst;

static void orc_reserve(orc_inst* s, int64_t want)
{
    if (want <= s->cap) return;
    int64_t cap = s->cap ? s->cap : 1024;
    while (cap < want) cap *= 2;
    s->x = (double*)realloc(s->x, sizeof(double) * 3 * cap);
    s->x0 = (double*)realloc(s->x0, sizeof(double) * 3 * cap);
    s->sp = (int32_t*)realloc(s->sp, sizeof(int32_t) * cap);
    s->uid = (uint64_t*)realloc(s->uid, sizeof(uint64_t) * cap);
    s->cap = cap;
}

orc_inst* orc_new(double L, uint64_t seed, uint64_t inst)
{
    orc_inst* s = (orc_inst*)calloc(1, sizeof(orc_inst));
    s->L = L;
    s->key[0] = seed;
    s->key[1] = inst;
    orc_reserve(s, 1024);
    return s;
}

void orc_free(orc_inst* s)
{
    if (!s) return;
    free(s->x); free(s->x0); free(s->sp); free(s->uid);
    free(s->log_uid); free(s->log_P); free(s->log_u24); free(s->log_flag); free(s->log_rx);
    free(s);
}

int64_t orc_get_n(const orc_inst* s) { return s->n; }
int64_t orc_get_step(const orc_inst* s) { return s->step; }
double orc_get_time(const orc_inst* s) { return s->t; }
double orc_get_edep(const orc_inst* s) { return s->edep_eV; }
void orc_get_diag(const orc_inst* s, int64_t out[3])
{
    out[0] = s->n_cand; out[1] = s->n_acc; out[2] = s->n_react;
}

/* Append molecules (positions already inside the cube) with fresh uids taken
 * in array order from the instance's uid counter; start position = position. */
void orc_inject(orc_inst* s, int64_t n, const double* xyz, const int32_t* sp, double edep_eV)
{
    orc_reserve(s, s->n + n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = s->n + i;
        for (int a = 0; a < 3; ++a) {
            s->x[3 * k + a] = orc_wrap(xyz[3 * i + a], s->L);
            s->x0[3 * k + a] = s->x[3 * k + a];
        }
        s->sp[k] = sp[i];
        s->uid[k] = s->next_uid++;
    }
    s->n += n;
    s->edep_eV += edep_eV;
}

/* Replace the whole state (debug and parity tests). */
void orc_set_state(orc_inst* s, int64_t n, const double* xyz, const double* x0, const int32_t* sp,
                   const uint64_t* uid, int64_t step, uint64_t next_uid)
{
    s->n = 0;
    orc_reserve(s, n);
    memcpy(s->x, xyz, sizeof(double) * 3 * n);
    memcpy(s->x0, x0 ? x0 : xyz, sizeof(double) * 3 * n);
    memcpy(s->sp, sp, sizeof(int32_t) * n);
    memcpy(s->uid, uid, sizeof(uint64_t) * n);
    s->n = n;
    s->step = step;
    s->next_uid = next_uid;
}

void orc_get_state(const orc_inst* s, double* xyz, double* x0, int32_t* sp, uint64_t* uid)
{
    if (xyz) memcpy(xyz, s->x, sizeof(double) * 3 * s->n);
    if (x0) memcpy(x0, s->x0, sizeof(double) * 3 * s->n);
    if (sp) memcpy(sp, s->sp, sizeof(int32_t) * s->n);
    if (uid) memcpy(uid, s->uid, sizeof(uint64_t) * s->n);
}

void orc_counts(const orc_inst* s, int32_t ns, int64_t* out)
{
    for (int32_t k = 0; k < ns; ++k) out[k] = 0;
    for (int64_t i = 0; i < s->n; ++i)
        if (s->sp[i] >= 0 && s->sp[i] < ns) out[s->sp[i]]++;
}

void orc_set_log(orc_inst* s, int32_t mode) { s->log_mode = mode; }
int64_t orc_log_size(const orc_inst* s) { return s->log_n; }
void orc_get_log(const orc_inst* s, uint64_t* uid2, double* P, uint32_t* u24, int32_t* flag, int32_t* rx)
{
    int64_t n = s->log_n;
    if (uid2) memcpy(uid2, s->log_uid, sizeof(uint64_t) * 2 * n);
    if (P) memcpy(P, s->log_P, sizeof(double) * n);
    if (u24) memcpy(u24, s->log_u24, sizeof(uint32_t) * n);
    if (flag) memcpy(flag, s->log_flag, sizeof(int32_t) * n);
    if (rx) memcpy(rx, s->log_rx, sizeof(int32_t) * n);
}

static void orc_log_push(orc_inst* s, uint64_t lo, uint64_t hi, double P, uint32_t u24, int32_t flag, int32_t rx)
{
    if (s->log_n == s->log_cap) {
        s->log_cap = s->log_cap ? 2 * s->log_cap : 1024;
        s->log_uid = (uint64_t*)realloc(s->log_uid, sizeof(uint64_t) * 2 * s->log_cap);
        s->log_P = (double*)realloc(s->log_P, sizeof(double) * s->log_cap);
        s->log_u24 = (uint32_t*)realloc(s->log_u24, sizeof(uint32_t) * s->log_cap);
        s->log_flag = (int32_t*)realloc(s->log_flag, sizeof(int32_t) * s->log_cap);
        s->log_rx = (int32_t*)realloc(s->log_rx, sizeof(int32_t) * s->log_cap);
    }
    int64_t k = s->log_n++;
    s->log_uid[2 * k] = lo;
    s->log_uid[2 * k + 1] = hi;
    s->log_P[k] = P;
    s->log_u24[k] = u24;
    s->log_flag[k] = flag;
    s->log_rx[k] = rx;
}

/* accepted pair */
typedef struct { int64_t i, j; uint32_t u24; int32_t rx; int64_t log_idx; } orc_pair;

typedef struct {
    orc_pair* p;
    int64_t n, cap;
} orc_pairs;

static void orc_pairs_push(orc_pairs* v, orc_pair q)
{
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 256;
        v->p = (orc_pair*)realloc(v->p, sizeof(orc_pair) * v->cap);
    }
    v->p[v->n++] = q;
}

typedef struct {
    int32_t rmap[ORC_MAX_SPECIES][ORC_MAX_SPECIES];
    double R[ORC_MAX_REACT], Dab[ORC_MAX_REACT], rc[ORC_MAX_REACT];
} orc_rtab;

static void orc_make_rtab(const orc_chem* c, double dt, orc_rtab* t)
{
    for (int a = 0; a < ORC_MAX_SPECIES; ++a)
        for (int b = 0; b < ORC_MAX_SPECIES; ++b) t->rmap[a][b] = -1;
    for (int r = 0; r < c->nr; ++r) {
        t->rmap[c->ra[r]][c->rb[r]] = r;
        t->rmap[c->rb[r]][c->ra[r]] = r;
        t->Dab[r] = c->D[c->ra[r]] + c->D[c->rb[r]];
        t->R[r] = orc_radius(c->k_in[r], t->Dab[r]);
        t->rc[r] = orc_cutoff(t->R[r], t->Dab[r], dt, c->c_cut);
    }
}

/* Test one unordered pair: is it a candidate (end separation below the
 * cutoff), and if so is the reaction accepted this step? */
static void orc_test_pair(orc_inst* s, const orc_chem* c, const orc_rtab* t, double dt,
                          int64_t i, int64_t j, orc_pairs* acc)
{
    int32_t rx = t->rmap[s->sp[i]][s->sp[j]];
    if (rx < 0) return;
    double L = s->L;
    double d1[3], d0[3];
    for (int a = 0; a < 3; ++a) {
        d1[a] = orc_minimg(s->x[3 * j + a] - s->x[3 * i + a], L);
        d0[a] = orc_minimg(s->x0[3 * j + a] - s->x0[3 * i + a], L);
    }
    double r1 = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
    if (r1 >= t->rc[rx]) return;
    s->n_cand++;
    double r0 = sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]);
    double R = t->R[rx];
    double P;
    if (c->contact_only) P = (r0 <= R || r1 <= R) ? 1.0 : 0.0;
    else P = orc_bridge(r0, r1, R, t->Dab[rx] * dt);
    uint64_t lo = s->uid[i] < s->uid[j] ? s->uid[i] : s->uid[j];
    uint64_t hi = s->uid[i] < s->uid[j] ? s->uid[j] : s->uid[i];
    uint64_t ctr[4] = {lo, hi, (uint64_t)s->step, 1}, w[4];
    orc_philox4x64_10(ctr, s->key, w);
    uint32_t u24 = (uint32_t)(w[0] >> 40);
    int accepted = orc_u24(w[0]) < P;
    int64_t li = -1;
    if (s->log_mode == 2 || (s->log_mode == 1 && accepted)) {
        li = s->log_n;
        orc_log_push(s, lo, hi, P, u24, accepted ? 1 : 0, rx);
    }
    if (accepted) {
        orc_pair q = {i, j, u24, rx, li};
        orc_pairs_push(acc, q);
        s->n_acc++;
    }
}

/* Matching key: the pair uniform, then the partner's uid (low 40 bits). */
static uint64_t orc_key(uint32_t u24, uint64_t partner_uid)
{
    return ((uint64_t)u24 << 40) | (partner_uid & 0xFFFFFFFFFFULL);
}

/* Single-partner matching of one step's accepted pairs.  Reading (the
 * paper's "reacts when within R" gives no rule for a molecule with several
 * accepted partners): each molecule's best accepted partner is the one with
 * the smallest key (pair uniform's 24-bit integer, then the partner's uid,
 * orc_key); pairs whose two molecules are each other's best react; the same
 * is repeated on the molecules still unmatched, over the pairs left, for at
 * most `rounds` rounds.  Pair k joins molecules pi[k] and pj[k] (indices below
 * n) with uniform u24[k]; uid[] holds the molecules' uids.  partner[m]
 * receives m's partner or -1; order[] (may be NULL) the matched pair indices
 * in the order they matched.  Returns the number of matched pairs, or
 * -(that number) - 1 if some molecule was matched twice in one round, which
 * needs two of its pairs with identical keys. */
int64_t orc_match(int64_t n, int64_t n_pairs, const int64_t* pi, const int64_t* pj, const uint32_t* u24,
                  const uint64_t* uid, int32_t rounds, int64_t* partner, int64_t* order)
{
    uint64_t* best = (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1));
    int64_t* got = order ? order : (int64_t*)malloc(sizeof(int64_t) * (n_pairs ? n_pairs : 1));
    int64_t n_matched = 0;
    int tie = 0;
    for (int64_t i = 0; i < n; ++i) partner[i] = -1;
    for (int round = 0; round < rounds; ++round) {
        for (int64_t k = 0; k < n_pairs; ++k) {
            best[pi[k]] = UINT64_MAX;
            best[pj[k]] = UINT64_MAX;
        }
        for (int64_t k = 0; k < n_pairs; ++k) {
            if (partner[pi[k]] >= 0 || partner[pj[k]] >= 0) continue;
            uint64_t ki = orc_key(u24[k], uid[pj[k]]);
            uint64_t kj = orc_key(u24[k], uid[pi[k]]);
            if (ki < best[pi[k]]) best[pi[k]] = ki;
            if (kj < best[pj[k]]) best[pj[k]] = kj;
        }
        int64_t first = n_matched;
        for (int64_t k = 0; k < n_pairs; ++k) {
            if (partner[pi[k]] >= 0 || partner[pj[k]] >= 0) continue;
            if (best[pi[k]] == orc_key(u24[k], uid[pj[k]]) && best[pj[k]] == orc_key(u24[k], uid[pi[k]]))
                got[n_matched++] = k;
        }
        for (int64_t m = first; m < n_matched; ++m) {
            int64_t k = got[m];
            if (partner[pi[k]] >= 0 || partner[pj[k]] >= 0) tie = 1;
            partner[pi[k]] = pj[k];
            partner[pj[k]] = pi[k];
        }
        if (n_matched == first) break;
    }
    free(best);
    if (!order) free(got);
    return tie ? -n_matched - 1 : n_matched;
}

/* One SBS step of length dt.  Returns the number of reactions, or -1 if two
 * pairs sharing a molecule carried identical matching keys (never expected). */
int64_t orc_step(orc_inst* s, const orc_chem* c, double dt)
{
    const double L = s->L;
    const int64_t n = s->n;
    orc_rtab t;
    orc_make_rtab(c, dt, &t);
    s->n_cand = s->n_acc = s->n_react = 0;
    s->log_n = 0;

    /* 1. Brownian jump of every molecule (Gaussian of variance 2 D dt per
     *    axis), Philox counter (uid, step, 0, 0); then PBC 1, Eq. (1). */
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ctr[4] = {s->uid[i], (uint64_t)s->step, 0, 0}, w[4];
        double z[3];
        orc_philox4x64_10(ctr, s->key, w);
        orc_gauss3(w, z);
        double sigma = sqrt(2.0 * c->D[s->sp[i]] * dt);
        for (int a = 0; a < 3; ++a) {
            s->x0[3 * i + a] = s->x[3 * i + a];
            s->x[3 * i + a] = orc_wrap(s->x[3 * i + a] + sigma * z[a], L);
        }
    }

    /* 2. Candidate pairs and their acceptance. */
    orc_pairs acc = {0, 0, 0};
    double rcmax = 0.0;
    for (int r = 0; r < c->nr; ++r) if (t.rc[r] > rcmax) rcmax = t.rc[r];
    int64_t nc = (rcmax > 0.0) ? (int64_t)floor(L / rcmax) : 1;
    int64_t nc_occ = (int64_t)cbrt((double)n) + 1; /* larger buckets are always valid */
    if (nc > nc_occ) nc = nc_occ;
    if (c->brute || nc < 3) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) orc_test_pair(s, c, &t, dt, i, j, &acc);
    } else {
        /* bucket grid of edge h = L/nc >= rcmax: every candidate lies in one of
         * the 27 neighbouring buckets; each unordered pair is taken once (i<j). */
        int64_t ncell = nc * nc * nc;
        int64_t* head = (int64_t*)malloc(sizeof(int64_t) * ncell);
        int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
        int64_t* cidx = (int64_t*)malloc(sizeof(int64_t) * 3 * (n ? n : 1));
        for (int64_t k = 0; k < ncell; ++k) head[k] = -1;
        for (int64_t i = 0; i < n; ++i) {
            int64_t ci[3];
            for (int a = 0; a < 3; ++a) {
                int64_t q = (int64_t)floor((s->x[3 * i + a] + 0.5 * L) / L * (double)nc);
                if (q < 0) q = 0;
                if (q >= nc) q = nc - 1;
                ci[a] = q;
                cidx[3 * i + a] = q;
            }
            int64_t cell = (ci[0] * nc + ci[1]) * nc + ci[2];
            next[i] = head[cell];
            head[cell] = i;
        }
        for (int64_t i = 0; i < n; ++i) {
            for (int ox = -1; ox <= 1; ++ox)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int oz = -1; oz <= 1; ++oz) {
                        int64_t qx = (cidx[3 * i] + ox + nc) % nc;
                        int64_t qy = (cidx[3 * i + 1] + oy + nc) % nc;
                        int64_t qz = (cidx[3 * i + 2] + oz + nc) % nc;
                        for (int64_t j = head[(qx * nc + qy) * nc + qz]; j >= 0; j = next[j])
                            if (j > i) orc_test_pair(s, c, &t, dt, i, j, &acc);
                    }
        }
        free(head); free(next); free(cidx);
    }

    /* 3. Single-partner matching (orc_match). */
    int64_t* partner = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t* matched_pairs = (int64_t*)malloc(sizeof(int64_t) * (acc.n ? acc.n : 1));
    int64_t* mi = (int64_t*)malloc(sizeof(int64_t) * (acc.n ? acc.n : 1));
    int64_t* mj = (int64_t*)malloc(sizeof(int64_t) * (acc.n ? acc.n : 1));
    uint32_t* mu = (uint32_t*)malloc(sizeof(uint32_t) * (acc.n ? acc.n : 1));
    for (int64_t k = 0; k < acc.n; ++k) { mi[k] = acc.p[k].i; mj[k] = acc.p[k].j; mu[k] = acc.p[k].u24; }
    int64_t n_matched = orc_match(n, acc.n, mi, mj, mu, s->uid, c->rounds, partner, matched_pairs);
    int tie = n_matched < 0;
    if (tie) n_matched = -n_matched - 1;
    free(mi); free(mj); free(mu);

    /* 4. Reactions (Table 1).  Reading: products sit at the D-weighted point
     *    x_a + D_a/(D_a+D_b) * minimg(x_b - x_a) (a = reactant with the lower
     *    uid), wrapped; product 1 keeps uid_a, product 2 keeps uid_b, a third
     *    product takes a Philox word (counter (uid_a, uid_b, step, 2)) with the
     *    top bit set.  Products start the next step at rest (x0 = x). */
    int64_t nprod_total = 0;
    for (int64_t m = 0; m < n_matched; ++m) nprod_total += c->nprod[acc.p[matched_pairs[m]].rx];
    double* px = (double*)malloc(sizeof(double) * 3 * (nprod_total ? nprod_total : 1));
    int32_t* psp = (int32_t*)malloc(sizeof(int32_t) * (nprod_total ? nprod_total : 1));
    uint64_t* puid = (uint64_t*)malloc(sizeof(uint64_t) * (nprod_total ? nprod_total : 1));
    char* dead = (char*)calloc((size_t)(n ? n : 1), 1);
    int64_t np = 0;
    for (int64_t m = 0; m < n_matched; ++m) {
        orc_pair q = acc.p[matched_pairs[m]];
        int32_t rx = q.rx;
        if (q.log_idx >= 0) s->log_flag[q.log_idx] |= 2;
        int64_t a = q.i, b = q.j;
        if (s->uid[b] < s->uid[a]) { int64_t tmp = a; a = b; b = tmp; }
        if (c->keep_b[rx]) {
            /* the molecule of species rb stays where it is */
            int64_t keep = (s->sp[a] == c->rb[rx]) ? a : b;
            int64_t gone = (keep == a) ? b : a;
            dead[gone] = 1;
            continue;
        }
        dead[a] = dead[b] = 1;
        double Da = c->D[s->sp[a]], Db = c->D[s->sp[b]];
        double wgt = (Da + Db > 0.0) ? Da / (Da + Db) : 0.5;
        double xp[3];
        for (int k = 0; k < 3; ++k) {
            double d = orc_minimg(s->x[3 * b + k] - s->x[3 * a + k], L);
            xp[k] = orc_wrap(s->x[3 * a + k] + wgt * d, L);
        }
        for (int k = 0; k < c->nprod[rx]; ++k) {
            uint64_t u;
            if (k == 0) u = s->uid[a];
            else if (k == 1) u = s->uid[b];
            else {
                uint64_t ctr[4] = {s->uid[a], s->uid[b], (uint64_t)s->step, 2}, w[4];
                orc_philox4x64_10(ctr, s->key, w);
                u = w[0] | 0x8000000000000000ULL;
            }
            for (int e = 0; e < 3; ++e) px[3 * np + e] = xp[e];
            psp[np] = c->prod[rx][k];
            puid[np] = u;
            ++np;
        }
    }
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (dead[i]) continue;
        if (w != i) {
            for (int e = 0; e < 3; ++e) { s->x[3 * w + e] = s->x[3 * i + e]; s->x0[3 * w + e] = s->x0[3 * i + e]; }
            s->sp[w] = s->sp[i];
            s->uid[w] = s->uid[i];
        }
        ++w;
    }
    s->n = w;

    /* 5. First-order channels (extension).  Every molecule that survived the
     *    step's pair reactions (not this step's products) converts with
     *    probability p = 1 - exp(-k dt), decided by the top 24 bits k24 of
     *    word 0 of the Philox block at counter (uid, step, 3, 0): converts iff
     *    (2 k24 + 1) 2^-25 < p.  Product 1 takes the molecule's place and uid,
     *    product 2 appears at the same point (x0 = x) with uid = word 1 with
     *    the top bit set; no product removes the molecule. */
    int64_t n_fo2 = 0;
    for (int64_t i = 0; i < w; ++i) if (c->fo_k[s->sp[i]] > 0.0 && c->fo_nprod[s->sp[i]] == 2) ++n_fo2;
    double* fx = (double*)malloc(sizeof(double) * 3 * (n_fo2 ? n_fo2 : 1));
    int32_t* fsp = (int32_t*)malloc(sizeof(int32_t) * (n_fo2 ? n_fo2 : 1));
    uint64_t* fuid = (uint64_t*)malloc(sizeof(uint64_t) * (n_fo2 ? n_fo2 : 1));
    int64_t nf = 0;
    char* gone = (char*)calloc((size_t)(w ? w : 1), 1);
    for (int64_t i = 0; i < w; ++i) {
        const int32_t sp = s->sp[i];
        if (!(c->fo_k[sp] > 0.0)) continue;
        const double pc = -expm1(-c->fo_k[sp] * dt);
        uint64_t ctr[4] = {s->uid[i], (uint64_t)s->step, 3, 0}, wd[4];
        orc_philox4x64_10(ctr, s->key, wd);
        const double u = (double)(2 * (wd[0] >> 40) + 1) * (1.0 / 33554432.0);
        if (!(u < pc)) continue;
        if (c->fo_nprod[sp] == 0) { gone[i] = 1; continue; }
        s->sp[i] = c->fo_prod[sp][0];
        if (c->fo_nprod[sp] == 2) {
            for (int e = 0; e < 3; ++e) fx[3 * nf + e] = s->x[3 * i + e];
            fsp[nf] = c->fo_prod[sp][1];
            fuid[nf] = wd[1] | 0x8000000000000000ULL;
            ++nf;
        }
    }
    int64_t w2 = 0;
    for (int64_t i = 0; i < w; ++i) {
        if (gone[i]) continue;
        if (w2 != i) {
            for (int e = 0; e < 3; ++e) { s->x[3 * w2 + e] = s->x[3 * i + e]; s->x0[3 * w2 + e] = s->x0[3 * i + e]; }
            s->sp[w2] = s->sp[i];
            s->uid[w2] = s->uid[i];
        }
        ++w2;
    }
    w = w2;
    s->n = w;
    orc_reserve(s, w + nf);
    for (int64_t k = 0; k < nf; ++k) {
        for (int e = 0; e < 3; ++e) { s->x[3 * (w + k) + e] = fx[3 * k + e]; s->x0[3 * (w + k) + e] = fx[3 * k + e]; }
        s->sp[w + k] = fsp[k];
        s->uid[w + k] = fuid[k];
    }
    w += nf;
    s->n = w;
    free(fx); free(fsp); free(fuid); free(gone);
    orc_reserve(s, w + np);
    for (int64_t k = 0; k < np; ++k) {
        for (int e = 0; e < 3; ++e) { s->x[3 * (w + k) + e] = px[3 * k + e]; s->x0[3 * (w + k) + e] = px[3 * k + e]; }
        s->sp[w + k] = psp[k];
        s->uid[w + k] = puid[k];
    }
    s->n = w + np;
    s->n_react = n_matched;
    s->step++;
    s->t += dt;
    free(px); free(psp); free(puid); free(dead);
    free(partner); free(matched_pairs); free(acc.p);
    return tie ? -1 : n_matched;
}

/* ------------------------------------------------------------------------ */
/* Driver: injections at given times, steps from the schedule above, species */
/* counts at record times (injection first, then the record).  This is the   */
/* beam-on/beam-off alternation of Sec. "Workflow of gMicroMC extension"     */
/* with SBS in both phases.                                                  */
/* ------------------------------------------------------------------------ */
int64_t orc_run(orc_inst* s, const orc_chem* c,
                int32_t n_inj, const double* inj_t, const int64_t* inj_n, const double* inj_xyz,
                const int32_t* inj_sp, const double* inj_edep,
                int32_t n_rec, const double* rec_t, double t_end, double dt0, double ratio, double dt_max,
                int64_t* counts, double* edep_rec, int64_t* stats)
{
    int32_t ns = c->ns;
    int64_t* inj_off = (int64_t*)malloc(sizeof(int64_t) * (n_inj + 1));
    inj_off[0] = 0;
    for (int32_t k = 0; k < n_inj; ++k) inj_off[k + 1] = inj_off[k] + inj_n[k];
    double* events = (double*)malloc(sizeof(double) * (n_inj + n_rec + 1));
    int32_t n_ev = 0;
    for (int32_t k = 0; k < n_rec; ++k) events[n_ev++] = rec_t[k];
    for (int32_t k = 0; k < n_inj; ++k) events[n_ev++] = inj_t[k];
    int64_t nsteps = orc_schedule(s->t, t_end, n_inj, inj_t, n_ev, events, dt0, ratio, dt_max, NULL, 0);
    double* sched = (double*)malloc(sizeof(double) * (nsteps ? nsteps : 1));
    orc_schedule(s->t, t_end, n_inj, inj_t, n_ev, events, dt0, ratio, dt_max, sched, nsteps);

    int64_t msteps = 0, nreact = 0, bad = 0;
    int32_t next_inj = 0;
    /* boundary handler at the current time */
#define ORC_BOUNDARY()                                                                     \
    do {                                                                                   \
        while (next_inj < n_inj && inj_t[next_inj] <= s->t) {                              \
            orc_inject(s, inj_n[next_inj], inj_xyz + 3 * inj_off[next_inj],                \
                       inj_sp + inj_off[next_inj], inj_edep ? inj_edep[next_inj] : 0.0);   \
            ++next_inj;                                                                    \
        }                                                                                  \
        for (int32_t r = 0; r < n_rec; ++r)                                                \
            if (rec_t[r] == s->t) {                                                        \
                orc_counts(s, ns, counts + (int64_t)r * ns);                               \
                if (edep_rec) edep_rec[r] = s->edep_eV;                                    \
            }                                                                              \
    } while (0)

    ORC_BOUNDARY();
    for (int64_t k = 0; k < nsteps; ++k) {
        double te = sched[k];
        msteps += s->n;
        int64_t nr = orc_step(s, c, te - s->t);
        if (nr < 0) bad = 1; else nreact += nr;
        s->t = te; /* exact step end (avoid drift of t += dt) */
        ORC_BOUNDARY();
    }
#undef ORC_BOUNDARY
    if (stats) { stats[0] = nsteps; stats[1] = msteps; stats[2] = nreact; stats[3] = bad; }
    free(inj_off); free(events); free(sched);
    return nsteps;
}

/* ------------------------------------------------------------------------ */
/* Single-precision emulation of the integer decisions the engine takes in   */
/* FP32 (IEEE binary32, round to nearest even, no fused multiply-add).       */
/* ------------------------------------------------------------------------ */

/* Cell of each position for an nc^3 grid: i = min(nc-1, floor((x + L/2) * (nc/L)))
 * per axis, cell = (ix*nc + iy)*nc + iz. */
void orc_bin_f32(int64_t n, const float* xyz, float L, int32_t nc, int32_t* cell)
{
    volatile float halfL = 0.5f * L;
    volatile float inv_h = (float)nc / L;
    for (int64_t i = 0; i < n; ++i) {
        int32_t q[3];
        for (int a = 0; a < 3; ++a) {
            volatile float t = xyz[3 * i + a] + halfL;
            volatile float u = t * inv_h;
            int32_t k = (int32_t)floorf(u);
            if (k > nc - 1) k = nc - 1;
            if (k < 0) k = 0;
            q[a] = k;
        }
        cell[i] = (q[0] * nc + q[1]) * nc + q[2];
    }
}

/* Squared candidate cutoff of every reaction in FP32: (float)(rc*rc) with rc in FP64. */
void orc_rc2_f32(const orc_chem* c, double dt, float* out)
{
    for (int r = 0; r < c->nr; ++r) {
        double Dab = c->D[c->ra[r]] + c->D[c->rb[r]];
        double rc = orc_cutoff(orc_radius(c->k_in[r], Dab), Dab, dt, c->c_cut);
        out[r] = (float)(rc * rc);
    }
}

/* All candidate pairs (i<j) among float positions by brute force, FP32:
 * d = x_j - x_i, minimum image per Eq. (2), d2 = (dx*dx + dy*dy) + dz*dz,
 * candidate iff d2 < rc2.  Returns the count; writes up to max pairs. */
int64_t orc_cand_f32(int64_t n, const float* xyz, const int32_t* sp, float L, const orc_chem* c,
                     double dt, int64_t* pairs, int64_t max)
{
    float rc2[ORC_MAX_REACT];
    int32_t rmap[ORC_MAX_SPECIES][ORC_MAX_SPECIES];
    orc_rc2_f32(c, dt, rc2);
    for (int a = 0; a < ORC_MAX_SPECIES; ++a)
        for (int b = 0; b < ORC_MAX_SPECIES; ++b) rmap[a][b] = -1;
    for (int r = 0; r < c->nr; ++r) { rmap[c->ra[r]][c->rb[r]] = r; rmap[c->rb[r]][c->ra[r]] = r; }
    const float halfL = 0.5f * L;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            int32_t rx = rmap[sp[i]][sp[j]];
            if (rx < 0) continue;
            volatile float d[3];
            for (int a = 0; a < 3; ++a) {
                volatile float v = xyz[3 * j + a] - xyz[3 * i + a];
                if (v >= halfL) v = v - L;
                else if (v < -halfL) v = v + L;
                d[a] = v;
            }
            volatile float sx = d[0] * d[0];
            volatile float sy = d[1] * d[1];
            volatile float sz = d[2] * d[2];
            volatile float s2 = sx + sy;
            volatile float d2 = s2 + sz;
            if (d2 < rc2[rx]) {
                if (cnt < max) { pairs[2 * cnt] = i; pairs[2 * cnt + 1] = j; }
                ++cnt;
            }
        }
    return cnt;
}

/* The FP32 candidate predicate of orc_cand_f32 for one pair (i < j). */
static int orc_is_cand_f32(const float* xyz, int64_t i, int64_t j, float L, float rc2)
{
    const float halfL = 0.5f * L;
    volatile float d[3];
    for (int a = 0; a < 3; ++a) {
        volatile float v = xyz[3 * j + a] - xyz[3 * i + a];
        if (v >= halfL) v = v - L;
        else if (v < -halfL) v = v + L;
        d[a] = v;
    }
    volatile float sx = d[0] * d[0];
    volatile float sy = d[1] * d[1];
    volatile float sz = d[2] * d[2];
    volatile float s2 = sx + sy;
    volatile float d2 = s2 + sz;
    return d2 < rc2;
}

/* One step's pair decisions on fixed FP32 positions, for inputs too large for
 * the all-pairs loop: the candidates are the pairs orc_cand_f32 selects (the
 * same FP32 predicate), found through a bucket grid of edge >= 1.001 x the
 * largest cutoff (27 neighbouring buckets, periodic), or all pairs when fewer
 * than 3 buckets fit; each candidate then gets the oracle's FP64 contact
 * probability (orc_bridge on the minimum-image separations of the end
 * positions xyz and the start positions xyz0) and its pair uniform (Philox at
 * (lower uid, higher uid, step, 1), key (seed, inst)), accepted iff u < P.
 * Writes up to max accepted pairs (sorted indices i < j, their P and u24);
 * returns the number accepted and the number of candidates in *n_cand. */
int64_t orc_accept_f32(int64_t n, const float* xyz, const float* xyz0, const int32_t* sp, const uint64_t* uid,
                       float L, const orc_chem* c, double dt, uint64_t step, uint64_t seed, uint64_t inst,
                       int64_t* pairs, double* P, uint32_t* u24, int64_t max, int64_t* n_cand)
{
    float rc2[ORC_MAX_REACT];
    int32_t rmap[ORC_MAX_SPECIES][ORC_MAX_SPECIES];
    orc_rc2_f32(c, dt, rc2);
    for (int a = 0; a < ORC_MAX_SPECIES; ++a)
        for (int b = 0; b < ORC_MAX_SPECIES; ++b) rmap[a][b] = -1;
    double rcmax = 0.0, R[ORC_MAX_REACT], Dab[ORC_MAX_REACT];
    for (int r = 0; r < c->nr; ++r) {
        rmap[c->ra[r]][c->rb[r]] = r;
        rmap[c->rb[r]][c->ra[r]] = r;
        Dab[r] = c->D[c->ra[r]] + c->D[c->rb[r]];
        R[r] = orc_radius(c->k_in[r], Dab[r]);
        double rc = sqrt((double)rc2[r]);
        if (rc > rcmax) rcmax = rc;
    }
    int64_t nc = (int64_t)floor((double)L / (1.001 * rcmax));
    if (nc > 256) nc = 256;
    const uint64_t key[2] = {seed, inst};
    int64_t n_acc = 0, cand = 0;
    /* candidate (i, j): evaluate and keep if accepted */
#define ORC_PAIR(I, J)                                                                         \
    do {                                                                                       \
        int64_t i_ = (I), j_ = (J);                                                            \
        int32_t rx = rmap[sp[i_]][sp[j_]];                                                     \
        if (rx >= 0 && orc_is_cand_f32(xyz, i_, j_, L, rc2[rx])) {                             \
            ++cand;                                                                            \
            double d1[3], d0[3];                                                               \
            for (int a = 0; a < 3; ++a) {                                                      \
                d1[a] = orc_minimg((double)xyz[3 * j_ + a] - (double)xyz[3 * i_ + a], L);      \
                d0[a] = orc_minimg((double)xyz0[3 * j_ + a] - (double)xyz0[3 * i_ + a], L);    \
            }                                                                                  \
            double r1 = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);                   \
            double r0 = sqrt(d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2]);                   \
            double p = c->contact_only ? ((r0 <= R[rx] || r1 <= R[rx]) ? 1.0 : 0.0)            \
                                       : orc_bridge(r0, r1, R[rx], Dab[rx] * dt);              \
            uint64_t lo = uid[i_] < uid[j_] ? uid[i_] : uid[j_];                               \
            uint64_t hi = uid[i_] < uid[j_] ? uid[j_] : uid[i_];                               \
            uint64_t ctr[4] = {lo, hi, step, 1}, w[4];                                         \
            orc_philox4x64_10(ctr, key, w);                                                    \
            if (orc_u24(w[0]) < p) {                                                           \
                if (n_acc < max) {                                                             \
                    pairs[2 * n_acc] = i_ < j_ ? i_ : j_;                                      \
                    pairs[2 * n_acc + 1] = i_ < j_ ? j_ : i_;                                  \
                    P[n_acc] = p;                                                              \
                    u24[n_acc] = (uint32_t)(w[0] >> 40);                                       \
                }                                                                              \
                ++n_acc;                                                                       \
            }                                                                                  \
        }                                                                                      \
    } while (0)
    if (nc < 3) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) ORC_PAIR(i, j);
    } else {
        int64_t ncell = nc * nc * nc;
        int64_t* head = (int64_t*)malloc(sizeof(int64_t) * ncell);
        int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
        int64_t* cid = (int64_t*)malloc(sizeof(int64_t) * 3 * (n ? n : 1));
        for (int64_t k = 0; k < ncell; ++k) head[k] = -1;
        for (int64_t i = n - 1; i >= 0; --i) {
            int64_t q[3];
            for (int a = 0; a < 3; ++a) {
                int64_t k = (int64_t)floor(((double)xyz[3 * i + a] + 0.5 * (double)L) / (double)L * (double)nc);
                q[a] = k < 0 ? 0 : (k >= nc ? nc - 1 : k);
                cid[3 * i + a] = q[a];
            }
            int64_t cell = (q[0] * nc + q[1]) * nc + q[2];
            next[i] = head[cell];
            head[cell] = i;
        }
        for (int64_t i = 0; i < n; ++i)
            for (int ox = -1; ox <= 1; ++ox)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int oz = -1; oz <= 1; ++oz) {
                        int64_t qx = (cid[3 * i] + ox + nc) % nc;
                        int64_t qy = (cid[3 * i + 1] + oy + nc) % nc;
                        int64_t qz = (cid[3 * i + 2] + oz + nc) % nc;
                        for (int64_t j = head[(qx * nc + qy) * nc + qz]; j >= 0; j = next[j])
                            if (j > i) ORC_PAIR(i, j);
                    }
        free(head); free(next); free(cid);
    }
#undef ORC_PAIR
    *n_cand = cand;
    return n_acc;
}

/* ------------------------------------------------------------------------ */
/* Homogeneous stochastic kinetics: Gillespie's direct method (Gillespie,    */
/* J. Phys. Chem. 81, 1977), the algorithm of the stochastic reference the   */
/* paper compares SBS + PBCs and its rate equations against (Sec. "Setup for  */
/* verification of periodic boundary conditions" and the discussion of the   */
/* PBC figure): the next reaction and the waiting time to it are drawn from   */
/* reaction probabilities built from the k list.                             */
/*                                                                          */
/* One well-mixed volume V (litres) holding integer counts n.  Reaction r    */
/* between species a and b has the stochastic constant c_r = k_r / (N_A V),  */
/* k_r = 10 k_in L/mol/ns (the printed value: 2k for a self-recombination),  */
/* and the propensity a_r = c_r h_r with h_r = n_a n_b (a != b) or           */
/* n_a (n_a - 1) / 2 (a == b), the number of distinct reactant pairs; this   */
/* is the stochastic form of the rate equations (event rate k[a][b], or      */
/* k[a]^2 / 2).  Each step: a_0 = sum of a_r in table order, waiting time    */
/* tau = -ln(u1) / a_0, reaction mu = the first r whose running sum of a_r   */
/* exceeds u2 a_0 (if rounding leaves none, the last r with a_r > 0), then   */
/* the reactants are removed (not b when keep_b) and the products added.     */
/* Extensions: the first-order channels of the chemistry (species order,    */
/* a = fo_k[s] n_s) and then the zero-order sources (R9's reverse, the water */
/* autoionisation; a_q = rate_q N_A V, rate in mol/L/ns) follow the          */
/* reactions in the propensity list.                                         */
/*                                                                          */
/* Random numbers: Philox4x64-10 with key (seed, 0x4753534153534131) and     */
/* counter (stream, j / 2, 0, 0) serve events j and j + 1 (j even): event j  */
/* takes u1, u2 from words 0 and 1, event j + 1 from words 2 and 3;          */
/* u = (top 53 bits + 1/2) 2^-53, in (0, 1).                                 */
/*                                                                          */
/* out[k][s] = the counts after every event at a time <= t_rec[k] (t_rec     */
/* ascending, times in ns from the start).  The run stops once the last      */
/* record is taken or no reaction can happen.  Returns the number of events, */
/* or -1 when max_events were taken before the last record.  ev_t / ev_r     */
/* (may be NULL) receive the time and reaction of the first ev_cap events.   */
/* ------------------------------------------------------------------------ */
static double orc_u53(uint64_t w)
{
    return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

int64_t orc_ssa(const orc_chem* c, double volume_L, const int64_t* n0, int32_t n_rec, const double* t_rec,
                uint64_t seed, uint64_t stream, int64_t max_events, int64_t* out, double* ev_t, int32_t* ev_r,
                int64_t ev_cap, int32_t n_src, const double* src_rate, const int32_t* src_nprod,
                const int32_t* src_prod)
{
    const double NA = 6.02214076e23;
    int64_t n[ORC_MAX_SPECIES];
    double cr[ORC_MAX_REACT], a[ORC_MAX_REACT + ORC_MAX_SPECIES + 8];
    int32_t fo_sp[ORC_MAX_SPECIES];
    int nfo = 0;
    for (int sp = 0; sp < c->ns; ++sp)
        if (c->fo_k[sp] > 0.0) fo_sp[nfo++] = sp;
    for (int s = 0; s < c->ns; ++s) n[s] = n0[s];
    for (int r = 0; r < c->nr; ++r) cr[r] = (10.0 * c->k_in[r]) / (NA * volume_L);
    if (n_src > 8) return -2;
    const uint64_t key[2] = {seed, 0x4753534153534131ULL};
    double t = 0.0;
    int64_t j = 0;
    int32_t rec = 0;
    uint64_t w[4] = {0, 0, 0, 0};
    for (;;) {
        double a0 = 0.0;
        for (int r = 0; r < c->nr; ++r) {
            const int64_t na = n[c->ra[r]], nb = n[c->rb[r]];
            const int64_t h = c->ra[r] == c->rb[r] ? na * (na - 1) / 2 : na * nb;
            a[r] = cr[r] * (double)h;
            a0 += a[r];
        }
        for (int q = 0; q < nfo; ++q) {
            a[c->nr + q] = c->fo_k[fo_sp[q]] * (double)n[fo_sp[q]];
            a0 += a[c->nr + q];
        }
        for (int q = 0; q < n_src; ++q) {
            a[c->nr + nfo + q] = src_rate[q] * (NA * volume_L);
            a0 += a[c->nr + nfo + q];
        }
        double t_next = INFINITY, u2 = 0.0;
        if (a0 > 0.0) {
            if ((j & 1) == 0) {
                const uint64_t ctr[4] = {stream, (uint64_t)j >> 1, 0, 0};
                orc_philox4x64_10(ctr, key, w);
            }
            const uint64_t* wj = w + 2 * (j & 1);
            t_next = t + (-log(orc_u53(wj[0])) / a0);
            u2 = orc_u53(wj[1]);
        }
        while (rec < n_rec && t_rec[rec] < t_next) {
            for (int s = 0; s < c->ns; ++s) out[(int64_t)rec * c->ns + s] = n[s];
            ++rec;
        }
        if (rec == n_rec) return j;
        if (j == max_events) return -1;
        const double target = u2 * a0;
        double cum = 0.0;
        int mu = -1, last = -1;
        for (int r = 0; r < c->nr + nfo + n_src; ++r) {
            cum += a[r];
            if (a[r] > 0.0) last = r;
            if (target < cum) { mu = r; break; }
        }
        if (mu < 0) mu = last;
        if (mu < c->nr) {
            n[c->ra[mu]] -= 1;
            if (!c->keep_b[mu]) n[c->rb[mu]] -= 1;
            for (int k = 0; k < c->nprod[mu]; ++k) n[c->prod[mu][k]] += 1;
        } else if (mu < c->nr + nfo) {
            const int sp = fo_sp[mu - c->nr];
            n[sp] -= 1;
            for (int k = 0; k < c->fo_nprod[sp]; ++k) n[c->fo_prod[sp][k]] += 1;
        } else {
            const int q = mu - c->nr - nfo;
            for (int k = 0; k < src_nprod[q]; ++k) n[src_prod[3 * q + k]] += 1;
        }
        if (ev_t && j < ev_cap) { ev_t[j] = t_next; ev_r[j] = mu; }
        t = t_next;
        ++j;
    }
}

/* ------------------------------------------------------------------------ */
/* Counter-based spur model (input side: it stands in for the paper's       */
/* physical and physico-chemical stages, which are out of scope).  A pulse   */
/* of n_tracks straight tracks parallel to z through the cube; on each track */
/* spur centres at exponential spacing, a Poisson number of molecules per    */
/* spur, species drawn from fixed fractions, Gaussian offsets per axis.      */
/* Philox4x64-10, key (seed, 0x53505552534D4F44), u = (top 53 bits + 1/2)    */
/* 2^-53:                                                                   */
/*   track k, block (stream, k, 0, 0): x = -L/2 + L u0, y = -L/2 + L u1;     */
/*   spur j, block (stream, k, j + 1, 0): z_j = z_{j-1} - spacing ln u0      */
/*     (z_{-1} = -L/2; the track ends at the first z_j >= L/2), molecule     */
/*     count by inversion of the Poisson CDF at u1 (at most 64);            */
/*   molecule m, block (stream, k, j + 1, 2m + 1): offsets                  */
/*     sigma sqrt(-2 ln u0) (cos, sin)(2 pi u1) on x, y and                 */
/*     sigma sqrt(-2 ln u2) cos(2 pi u3) on z; block (stream, k, j + 1,     */
/*     2m + 2): species = first s with u0 < frac_0 + ... + frac_s (the last  */
/*     species with a positive fraction otherwise).                          */
/* Positions are wrapped into [-L/2, L/2).  Writes up to cap molecules in   */
/* track, spur, molecule order and returns how many the pulse has.           */
/* ------------------------------------------------------------------------ */
int64_t orc_spurs(double L, uint64_t seed, uint64_t stream, int32_t n_tracks, double spacing, double mean,
                  double sigma, int32_t ns, const double* frac, double* xyz, int32_t* sp, int64_t cap)
{
    const uint64_t key[2] = {seed, 0x53505552534D4F44ULL};
    const double two_pi = 6.283185307179586476925286766559;
    int last = 0;
    for (int s = 0; s < ns; ++s) if (frac[s] > 0.0) last = s;
    int64_t n = 0;
    for (int32_t k = 0; k < n_tracks; ++k) {
        uint64_t w[4];
        uint64_t ctr[4] = {stream, (uint64_t)k, 0, 0};
        orc_philox4x64_10(ctr, key, w);
        const double x = -0.5 * L + L * orc_u53(w[0]), y = -0.5 * L + L * orc_u53(w[1]);
        double z = -0.5 * L;
        for (uint64_t j = 0; j < (1u << 20); ++j) {
            uint64_t cj[4] = {stream, (uint64_t)k, j + 1, 0};
            orc_philox4x64_10(cj, key, w);
            z = z - spacing * log(orc_u53(w[0]));
            if (z >= 0.5 * L) break;
            const double u = orc_u53(w[1]);
            int cnt = 0;
            double p = exp(-mean), F = p;
            while (u > F && cnt < 64) { ++cnt; p *= mean / cnt; F += p; }
            for (int m = 0; m < cnt; ++m) {
                uint64_t cm[4] = {stream, (uint64_t)k, j + 1, (uint64_t)(2 * m + 1)}, v[4];
                orc_philox4x64_10(cm, key, v);
                const double r1 = sigma * sqrt(-2.0 * log(orc_u53(v[0])));
                const double a1 = two_pi * orc_u53(v[1]);
                const double r2 = sigma * sqrt(-2.0 * log(orc_u53(v[2])));
                const double a2 = two_pi * orc_u53(v[3]);
                cm[3] = (uint64_t)(2 * m + 2);
                orc_philox4x64_10(cm, key, v);
                const double us = orc_u53(v[0]);
                double cum = 0.0;
                int s_pick = last;
                for (int s = 0; s < ns; ++s) {
                    cum += frac[s];
                    if (us < cum) { s_pick = s; break; }
                }
                if (n < cap) {
                    xyz[3 * n + 0] = orc_wrap(x + r1 * cos(a1), L);
                    xyz[3 * n + 1] = orc_wrap(y + r1 * sin(a1), L);
                    xyz[3 * n + 2] = orc_wrap(z + r2 * cos(a2), L);
                    sp[n] = s_pick;
                }
                ++n;
            }
        }
    }
    return n;
}
