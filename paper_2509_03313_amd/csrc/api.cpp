// api.cpp -- C ABI (include/gsbs.h) and host scheduler of the SBS engine.
//
// The host decides, for every instance, the step end times (ramp after each
// injection, events, cap), builds the per-step parameter rows (sigma per
// species, cutoff, radius, search grid) in pinned memory, uploads them in
// chunks and launches the step kernels on the context's stream.  Injections
// and record copies are issued at the step boundaries they belong to.  No
// device result is needed on the host while stepping, so the stream is never
// drained inside gsbs_advance_to except at its end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "engine.h"
#include "gsbs.h"
#include "mlp.h"

using namespace gsbs;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

const char* const kBroken = "the context's state was lost by a failed gsbs_load; load a checkpoint or destroy it";

}  // namespace

// Error channel shared with the other ABI files (gsbs_last_error reads it).
int gsbs::set_error(int code, const char* msg) { return fail(code, msg); }

namespace {

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess)                                                                  \
            return fail(GSBS_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));            \
    } while (0)

constexpr int kChunk = 64;  // global steps per uploaded parameter chunk
constexpr int kFeatures = 7 + 9 * kSurBins + 1;  // surrogate input row

// 1e10 L/mol/s expressed per pair in nm^3/ns: 1e10 * 1e24 nm^3 / (N_A * 1e9 ns)
double rate_to_nm3_per_ns(double k_in) { return k_in * (1e25 / 6.02214076e23); }

// Steady-state Smoluchowski radius (supplement: k = 4 pi R D_AB N_A).
double smol_radius(double k_in, double Dab) {
    return rate_to_nm3_per_ns(k_in) / (4.0 * 3.14159265358979323846264338327950 * Dab);
}

double cutoff_of(double R, double Dab, double dt, double c) { return R + c * std::sqrt(2.0 * Dab * dt); }

struct Pending {
    double t;
    int64_t n;
    float* d_xyz;
    uint8_t* d_sp;
    double edep;
};

struct InstHost {
    double L = 0;
    int64_t cap_hint = 0;
    double t = 0;
    uint64_t step = 0;
    uint64_t next_uid = 0;
    double edep = 0;
    int64_t n_est = 0;
    int64_t sp_est[kMaxSpecies] = {};  // species counts at the last refresh
    std::vector<double> anchors;
    std::vector<Pending> pending;
    std::vector<double> rec_t;
    std::vector<char> rec_done;
    std::vector<double> rec_edep;
    double dt_max = 0;
    // surrogate hand-overs: estimates spent, the last hand-over point handled, log
    double sur_spent = 0;
    double sur_done = -INFINITY;
    struct Handover {
        double t_switch, t_next, estimate;
        int32_t taken;
    };
    std::vector<Handover> sur_log;
};

// The step schedule: lattice anchor + dt0 * ratio^j after every anchor up to the
// next one, every event a step end, lattice points within 1e-9 (relative) of
// an event dropped, gaps above dt_max split evenly.
struct TP {
    double t;
    int ev;
};

void plan_steps(double t_start, double t_end, const double* anchors, int na, const double* events, int ne,
                double dt0, double ratio, double dt_max, std::vector<double>& out) {
    std::vector<TP> pts;
    for (int k = 0; k < na; ++k) {
        const double a = anchors[k];
        const double nxt = (k + 1 < na) ? anchors[k + 1] : INFINITY;
        for (int64_t j = 0;; ++j) {
            const double p = a + dt0 * std::pow(ratio, (double)j);
            if (p >= nxt || p > t_end) break;
            if (p <= t_start) continue;
            pts.push_back({p, 0});
        }
    }
    for (int k = 0; k <= ne; ++k) {
        const double e = (k < ne) ? events[k] : t_end;
        if (!(e > t_start) || e > t_end) continue;
        pts.push_back({e, 1});
    }
    std::sort(pts.begin(), pts.end(), [](const TP& x, const TP& y) {
        if (x.t != y.t) return x.t < y.t;
        return x.ev > y.ev;
    });
    std::vector<TP> kept;
    kept.reserve(pts.size());
    for (const TP& q : pts) {
        const double prev = kept.empty() ? t_start : kept.back().t;
        const int prev_ev = kept.empty() ? 1 : kept.back().ev;
        if (q.t - prev <= 1e-9 * std::fabs(q.t)) {
            if (!kept.empty() && q.ev && !prev_ev) {
                kept.back() = q;
                continue;
            }
            if (!q.ev) continue;
            if (q.t == prev) continue;
        }
        kept.push_back(q);
    }
    out.clear();
    double prev = t_start;
    for (const TP& q : kept) {
        const double g = q.t - prev;
        if (g > dt_max) {
            const int64_t ns = (int64_t)std::ceil(g / dt_max);
            for (int64_t s = 1; s < ns; ++s) out.push_back(prev + g * (double)s / (double)ns);
        }
        out.push_back(q.t);
        prev = q.t;
    }
}

}  // namespace

struct gsbs_ctx {
    int n_inst = 0;
    uint64_t seed = 0;
    hipStream_t st = nullptr;
    std::vector<InstHost> inst;
    gsbs_params prm{};
    int ns = 0;
    std::vector<double> D;
    std::vector<gsbs_reaction> rx;
    std::vector<gsbs_source> src;  // zero-order sources (homogeneous solvers)
    std::vector<gsbs_first_order> fo;  // first-order channels, one per species at most
    std::vector<double> R;
    bool chem_ready = false;
    ChemDev chem_h{};
    ChemDev* chem_d = nullptr;

    int32_t cap = 0;
    float4* pos[2] = {nullptr, nullptr};
    uint64_t* uid[2] = {nullptr, nullptr};
    int cur = 0;
    float4* pos0 = nullptr;
    uint2* cellrank = nullptr;
    unsigned long long* claim = nullptr;
    int32_t* mate = nullptr;
    float4* x0_dbg = nullptr;
    float4* xnew = nullptr;
    int32_t cell_cap = 0;
    uint32_t* cell_count = nullptr;
    uint32_t* cell_start = nullptr;
    unsigned long long* scan_status = nullptr;
    uint32_t scan_epoch = 0;
    PairRec* pairs = nullptr;
    uint32_t pair_cap = 0;
    long long* counts = nullptr;
    unsigned long long* msteps = nullptr;
    DevCounters* ctr = nullptr;
    long long* rec = nullptr;
    int32_t max_rec = 0;

    hipEvent_t tune_ev[2 * kChunk] = {};
    // live-count estimate refreshed from lagged device counts while stepping
    long long* h_cnt[2] = {nullptr, nullptr};
    hipEvent_t cnt_ev[2] = {nullptr, nullptr};
    bool cnt_pending[2] = {false, false};
    std::vector<int64_t> cnt_mark[2];     // molecules injected per instance when the copy was queued
    std::vector<int64_t> injected;        // molecules injected per instance so far
    int cnt_slot = 0;
    InstStep* h_chunk[2] = {nullptr, nullptr};
    InstStep* d_chunk[2] = {nullptr, nullptr};
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};
    int chunk_buf = 0;

    int64_t steps = 0;
    int64_t max_live = 0;
    bool tuning = true;
    bool broken = false;  // a gsbs_load failed while replacing the state
    // surrogate hand-over (gsbs_set_surrogate)
    bool sur_on = false;
    gsbs_mlp* sur_net = nullptr;
    gsbs_surrogate sur_cfg{};
    std::vector<float> sur_mu, sur_sd, sur_lo, sur_hi, sur_mu_y, sur_sd_y;
    std::vector<double> sur_dt_edges, sur_c_edges, sur_table;
    float* sur_x = nullptr;  // [n_inst][296] feature rows of the instances at a hand-over point
    float* sur_y = nullptr;  // [n_inst][7] network outputs
    // profiling
    bool profiling = false;
    struct StepLog {
        int64_t step;
        double ms;
        int32_t nc, reach, by_species, cfg;
        int64_t n_est;
    };
    std::vector<StepLog> step_log;
    hipEvent_t prof_ev[2 * kStepKernels] = {};
    // live timing: events around the masked kernels of every step, one pool per
    // chunk buffer, read once the chunk's last kernel has finished (no drain)
    uint32_t live_mask = 0;
    std::vector<hipEvent_t> live_ev[2];
    hipEvent_t live_done[2] = {nullptr, nullptr};
    bool live_pending[2] = {false, false};
    int live_nstep[2] = {0, 0};
    int32_t live_flags[2][kChunk] = {};
    DevCounters live_base{};  // device counters when live timing was switched on
    int64_t live_bins = 0;    // bins scanned by the live-timed steps
    // executable graphs launched during the current advance (destroyed after its final sync)
    // executable step graphs kept for reuse: a captured chunk whose launches have
    // the shape of a cached one updates it (hipGraphExecUpdate) instead of
    // instantiating a new one; each entry's event marks the end of its last launch
    struct GraphEntry {
        hipGraphExec_t exec;
        hipEvent_t done;
        uint64_t uses;
    };
    std::vector<GraphEntry> graph_cache;
    int64_t graph_instantiated = 0, graph_updated = 0;
    // surrogate state buffers (allocated on first use)
    int32_t sur_cap = 0;
    int32_t* sur_ref_idx = nullptr;
    int32_t* sur_ref_cnt = nullptr;
    int32_t* sur_pair_ab = nullptr;
    float* sur_edges2 = nullptr;
    double* sur_shell = nullptr;
    unsigned long long* sur_hist = nullptr;
    float* sur_vec = nullptr;  // 3 x 296: mu, sd, and a staging row / network output
    long long* sur_newc = nullptr;
    double prof_ms[kStepKernels] = {};
    int64_t prof_n[kStepKernels] = {};
    int64_t prof_work[kStepKernels] = {};
    int64_t prof_cnd[kStepKernels] = {};
    unsigned long long prof_cand = 0;  // candidate counter at the last profiled step
    // last debug step
    int32_t dbg_nc = 0;
    int32_t dbg_cell_base = 0;
    int32_t dbg_by_species = 0;
};

namespace {

template <typename T>
int dalloc(T** p, size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T) + 16);
    if (e != hipSuccess) return fail(GSBS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    *p = (T*)q;
    return GSBS_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

#define CHK(x)                      \
    do {                            \
        int r_ = (x);               \
        if (r_ != GSBS_OK) return r_; \
    } while (0)

int read_counters(gsbs_ctx* c, DevCounters* out) {
    HIPCHK(hipMemcpyAsync(out, c->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return GSBS_OK;
}

// Grow the molecule arrays to hold at least `need` molecules.  Every new
// buffer is allocated before an old one is freed: on an allocation failure
// the context keeps its state.
int ensure_capacity(gsbs_ctx* c, int64_t need) {
    if (need <= c->cap) return GSBS_OK;
    int64_t nc = std::max<int64_t>({need, (int64_t)c->cap * 2, 4096});
    if (nc > (int64_t)0x7FFFFFF0) return fail(GSBS_ECAPACITY, "molecule capacity beyond 2^31");
    DevCounters h{};
    int32_t n_in = 0;
    if (c->ctr) {
        CHK(read_counters(c, &h));
        n_in = h.n_in;
    }
    float4* np[2] = {nullptr, nullptr};
    uint64_t* nu[2] = {nullptr, nullptr};
    float4 *npos0 = nullptr, *nx0 = nullptr, *nxnew = nullptr;
    uint2* ncr = nullptr;
    unsigned long long* ncl = nullptr;
    int32_t* nmate = nullptr;
    PairRec* npairs = nullptr;
    const uint32_t want_pairs = (uint32_t)std::max<int64_t>(1 << 16, nc);
    int rc = GSBS_OK;
    for (int b = 0; b < 2; ++b) {
        if (rc == GSBS_OK) rc = dalloc(&np[b], nc);
        if (rc == GSBS_OK) rc = dalloc(&nu[b], nc);
    }
    if (rc == GSBS_OK) rc = dalloc(&npos0, nc);
    if (rc == GSBS_OK) rc = dalloc(&ncr, nc);
    if (rc == GSBS_OK) rc = dalloc(&ncl, nc);
    if (rc == GSBS_OK) rc = dalloc(&nmate, nc);
    if (rc == GSBS_OK) rc = dalloc(&nx0, nc);
    if (rc == GSBS_OK) rc = dalloc(&nxnew, nc);
    if (rc == GSBS_OK && want_pairs > c->pair_cap) rc = dalloc(&npairs, want_pairs);
    hipError_t e = hipSuccess;
    if (rc == GSBS_OK && n_in > 0) {
        e = hipMemcpyAsync(np[0], c->pos[c->cur], sizeof(float4) * n_in, hipMemcpyDeviceToDevice, c->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(nu[0], c->uid[c->cur], sizeof(uint64_t) * n_in, hipMemcpyDeviceToDevice, c->st);
    }
    if (rc == GSBS_OK && e == hipSuccess) e = hipMemsetAsync(ncl, 0xFF, sizeof(unsigned long long) * nc, c->st);
    if (rc == GSBS_OK && e == hipSuccess) e = hipMemsetAsync(nmate, 0xFF, sizeof(int32_t) * nc, c->st);
    if (rc == GSBS_OK && e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (rc != GSBS_OK || e != hipSuccess) {
        for (int b = 0; b < 2; ++b) {
            dfree(np[b]);
            dfree(nu[b]);
        }
        dfree(npos0);
        dfree(ncr);
        dfree(ncl);
        dfree(nmate);
        dfree(nx0);
        dfree(nxnew);
        dfree(npairs);
        if (rc != GSBS_OK) return rc;
        return fail(GSBS_EHIP, std::string("growing the molecule arrays: ") + hipGetErrorString(e));
    }
    for (int b = 0; b < 2; ++b) {
        dfree(c->pos[b]);
        dfree(c->uid[b]);
        c->pos[b] = np[b];
        c->uid[b] = nu[b];
    }
    c->cur = 0;
    dfree(c->pos0);
    dfree(c->cellrank);
    dfree(c->claim);
    dfree(c->mate);
    dfree(c->x0_dbg);
    dfree(c->xnew);
    c->pos0 = npos0;
    c->cellrank = ncr;
    c->claim = ncl;
    c->mate = nmate;
    c->x0_dbg = nx0;
    c->xnew = nxnew;
    c->cap = (int32_t)nc;
    if (npairs) {
        dfree(c->pairs);
        c->pairs = npairs;
        c->pair_cap = want_pairs;
    }
    return GSBS_OK;
}

int ensure_cells(gsbs_ctx* c, int64_t total) {
    if (total <= c->cell_cap) return GSBS_OK;
    int64_t nc = std::max<int64_t>(total, (int64_t)c->cell_cap * 2);
    nc = std::max<int64_t>(nc, 4096);
    HIPCHK(hipStreamSynchronize(c->st));
    dfree(c->cell_count);
    dfree(c->cell_start);
    dfree(c->scan_status);
    CHK(dalloc(&c->cell_count, nc + 1));
    CHK(dalloc(&c->cell_start, nc + 1));
    CHK(dalloc(&c->scan_status, nc / 4096 + 2));
    HIPCHK(hipMemsetAsync(c->cell_count, 0, sizeof(uint32_t) * (nc + 1), c->st));
    HIPCHK(hipMemsetAsync(c->scan_status, 0, sizeof(unsigned long long) * (nc / 4096 + 2), c->st));
    c->cell_cap = (int32_t)nc;
    return GSBS_OK;
}

int ensure_pairs(gsbs_ctx* c, uint32_t want) {
    if (want <= c->pair_cap) return GSBS_OK;
    HIPCHK(hipStreamSynchronize(c->st));
    dfree(c->pairs);
    CHK(dalloc(&c->pairs, want));
    c->pair_cap = want;
    return GSBS_OK;
}

int build_chem(gsbs_ctx* c) {
    ChemDev& h = c->chem_h;
    std::memset(&h, 0, sizeof(h));
    for (int a = 0; a < kMaxSpecies; ++a)
        for (int b = 0; b < kMaxSpecies; ++b) h.rmap[a][b] = -1;
    for (int s = 0; s < c->ns; ++s) h.D[s] = (float)c->D[s];
    c->R.assign(c->rx.size(), 0.0);
    uint32_t mask = 0;
    for (size_t r = 0; r < c->rx.size(); ++r) {
        const gsbs_reaction& q = c->rx[r];
        h.rmap[q.a][q.b] = (int32_t)r;
        h.rmap[q.b][q.a] = (int32_t)r;
        h.nprod[r] = q.n_products;
        for (int k = 0; k < 3; ++k) h.prod[r][k] = q.products[k];
        h.keep_b[r] = q.keep_b;
        h.rb[r] = q.b;
        mask |= (1u << q.a) | (1u << q.b);
        h.pmask[std::min(q.a, q.b)] |= 1u << std::max(q.a, q.b);
        const double Dab = c->D[q.a] + c->D[q.b];
        c->R[r] = Dab > 0 ? smol_radius(q.k_in, Dab) : 0.0;
    }
    h.reactive_mask = mask;
    for (const gsbs_first_order& f : c->fo) {
        h.fo_mask |= 1u << f.a;
        h.fo_nprod[f.a] = f.n_products;
        for (int k = 0; k < 2; ++k) h.fo_prod[f.a][k] = k < f.n_products ? f.products[k] : -1;
    }
    h.n_species = c->ns;
    h.rounds = c->prm.rounds;
    h.contact_only = c->prm.contact_only;
    if (!c->chem_d) CHK(dalloc(&c->chem_d, 1));
    HIPCHK(hipMemcpyAsync(c->chem_d, &h, sizeof(ChemDev), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    // largest step keeping every cutoff below L/2 (minimum image unique)
    for (auto& in : c->inst) {
        double best = INFINITY;
        for (size_t r = 0; r < c->rx.size(); ++r) {
            const double Dab = c->D[c->rx[r].a] + c->D[c->rx[r].b];
            if (Dab <= 0) continue;
            const double room = (0.5 * in.L - c->R[r]) / c->prm.c_cut;
            if (room <= 0) return fail(GSBS_EMINIMAGE, "reaction radius reaches L/2");
            best = std::min(best, room * room / (2.0 * Dab));
        }
        if (c->prm.dt_max_ns > 0) best = std::min(best, c->prm.dt_max_ns);
        in.dt_max = best;
    }
    c->chem_ready = true;
    return GSBS_OK;
}

// Physics of one step for one instance: sigma per species, cutoffs, radii,
// bridge scale, culling radii.  Returns the largest cutoff.
double fill_physics(const gsbs_ctx* c, double L, uint64_t step, int idx, double dt, bool active, InstStep& S) {
    std::memset(&S, 0, sizeof(S));
    S.L = (float)L;
    S.halfL = 0.5f * S.L;
    S.invL = 1.0f / S.L;
    S.active = active ? 1 : 0;
    S.step = step;
    S.key0 = c->seed;
    S.key1 = (uint64_t)idx;
    double rcmax = 0.0;
    if (!active) return 0.0;
    for (int s = 0; s < c->ns; ++s) S.sigma[s] = (float)std::sqrt(2.0 * c->D[s] * dt);
    for (const gsbs_first_order& f : c->fo) S.fo_p[f.a] = -std::expm1(-f.k_per_ns * dt);
    for (size_t r = 0; r < c->rx.size(); ++r) {
        const gsbs_reaction& q = c->rx[r];
        const double Dab = c->D[q.a] + c->D[q.b];
        const double rc = cutoff_of(c->R[r], Dab, dt, c->prm.c_cut);
        S.rc2[r] = (float)(rc * rc);
        S.R[r] = (float)c->R[r];
        S.inv_s[r] = (Dab * dt > 0) ? (float)(1.0 / (Dab * dt)) : 0.0f;
        const float cull = (float)(rc * (1.0 + 1e-4) * rc * (1.0 + 1e-4));
        S.cull2[r] = cull;
        const int lo = std::min(q.a, q.b), hi = std::max(q.a, q.b);
        S.cull2_sp[lo] = std::max(S.cull2_sp[lo], cull);
        S.cull2_all[lo] = std::max(S.cull2_all[lo], cull);
        S.cull2_all[hi] = std::max(S.cull2_all[hi], cull);
        rcmax = std::max(rcmax, rc);
    }
    return rcmax;
}

constexpr double kGridMargin = 1.0 + 1e-5;  // cells a little wider than cutoff/reach (FP32 binning)

// Search-grid configurations the autotuner chooses from: search mode, cells
// per cutoff when the cutoff sets the grid, target molecules per cell.
struct GridCfg {
    int by_species;
    int reach;
    double occ;
};
constexpr GridCfg kCfgs[] = {
    {0, 1, 2.0}, {0, 1, 6.0}, {0, 2, 2.0}, {1, 1, 16.0}, {1, 2, 16.0}, {1, 2, 64.0}, {1, 3, 16.0},
    {1, 3, 4.0}, {1, 3, 1.0}, {1, 4, 1.0},
};
constexpr int kNumCfg = (int)(sizeof(kCfgs) / sizeof(kCfgs[0]));

// A boxes of species s in the species-bin search grid of one instance.
int64_t boxes_of(const InstStep& S, int s) {
    const int kx = S.kdim_sp[s] & 0xFF, ky = (S.kdim_sp[s] >> 8) & 0xFF, kz = (S.kdim_sp[s] >> 16) & 0xFF;
    const int64_t nc = S.nc;
    return ((nc + kx - 1) / kx) * ((nc + ky - 1) / ky) * ((nc + kz - 1) / kz);
}

// Waves of the species-bin search resident on the device at once (its LDS
// and register use allow four 4-wave blocks per compute unit).
constexpr double kResidentWaves = 256.0 * 16.0;

// Stream slices of the species-bin search for one step over all instances:
// a box whose partner stream exceeds W = (the step's whole streamed work) /
// (4 x resident waves) is cut into ceil(work / W) slices (at most 64, at
// least 4 stages of 64 molecules each), so that no slice is longer than a
// quarter of a resident wave's share and long streams do not leave the
// device idle at the end of the launch.  Rewrites each row's work-item
// offsets; inactive rows get none.
void assign_splits(const gsbs_ctx* c, InstStep* rows, int n) {
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        const InstStep& S = rows[i];
        if (!S.active || !S.by_species) continue;
        for (int s = 0; s < c->ns; ++s)
            if (S.pm_dir[s]) total += (double)boxes_of(S, s) * (double)S.work_sp[s];
    }
    const double W = std::max(256.0, total / (4.0 * kResidentWaves));
    for (int i = 0; i < n; ++i) {
        InstStep& S = rows[i];
        if (!S.by_species) continue;
        int64_t off = 0;
        for (int s = 0; s < c->ns; ++s) {
            int64_t ns = 1;
            if (S.work_sp[s] > W) ns = std::min<int64_t>(64, (int64_t)std::ceil((double)S.work_sp[s] / W));
            ns = std::min<int64_t>(ns, std::max<int64_t>(1, (int64_t)(S.work_sp[s] / 256.0)));
            if (c->prm.search_split > 0) ns = c->prm.search_split;
            S.nsplit_sp[s] = (int32_t)ns;
            S.unit_off_sp[s] = (int32_t)off;
            if (S.active && S.pm_dir[s]) off += boxes_of(S, s) * ns;
        }
        S.unit_off_sp[c->ns] = (int32_t)std::min<int64_t>(off, 0x7FFFFFF0);
    }
}

// Grid of one instance for one configuration: nc cells per axis, no smaller
// than (cutoff / reach) and at least `occ` molecules per cell on average.
// Returns cells.
int32_t fill_grid(const gsbs_ctx* c, const int64_t* sp_est, double L, int64_t n_est, double rcmax, const GridCfg& g,
                  int32_t nc_force, InstStep& S) {
    int64_t nc;
    const int64_t nocc = std::max<int64_t>(1, (int64_t)std::floor(std::cbrt((double)std::max<int64_t>(n_est, 1) / g.occ)));
    if (nc_force > 0) {
        nc = nc_force;
    } else if (rcmax <= 0) {
        nc = nocc;
    } else {
        const int64_t ncr = std::max<int64_t>(1, (int64_t)std::floor(g.reach * L / (rcmax * kGridMargin)));
        nc = std::min<int64_t>(ncr, nocc);
    }
    nc = std::min<int64_t>(std::max<int64_t>(nc, 1), 1024);
    S.nc = (int32_t)nc;
    S.inv_h = (float)S.nc / S.L;
    S.h = S.L / (float)S.nc;
    S.reach = rcmax > 0 ? std::max(1, (int32_t)std::ceil(rcmax * kGridMargin * (double)nc / L)) : 1;
    // slack of the FP32 cell-distance bound: a few ulps of the edge plus the binning rounding
    S.cull_eps = 8.0f * std::nextafter(S.halfL, 2.0f * S.halfL) - 8.0f * S.halfL + 1e-6f * S.h;
    S.by_species = g.by_species;
    if (g.by_species) {
        // each pair of species is searched from the more abundant one (full waves)
        for (size_t r = 0; r < c->rx.size(); ++r) {
            const int a = c->rx[r].a, b = c->rx[r].b;
            if (a == b) {
                S.pm_dir[a] |= 1u << a;
            } else if (sp_est[a] > sp_est[b] || (sp_est[a] == sp_est[b] && a < b)) {
                S.pm_dir[a] |= 1u << b;
            } else {
                S.pm_dir[b] |= 1u << a;
            }
        }
        // A box of each species: kx*ky*kz cells chosen to minimise the partner
        // molecules streamed per A molecule (64 A molecules per wave pass, a fixed
        // cost per pass)
        const double ncell = (double)nc * nc * nc;
        for (int s = 0; s < c->ns; ++s) {
            S.kdim_sp[s] = 1 | (1 << 8) | (1 << 16);
            S.work_sp[s] = 0.0f;
            if (!S.pm_dir[s]) continue;
            const double per_cell = (double)std::max<int64_t>(sp_est[s], 0) / ncell;
            double best = INFINITY, best_work = 0.0;
            const int kmax = (int)std::min<int64_t>(nc, 8), kzmax = (int)std::min<int64_t>(nc, 16);
            double rho[kMaxSpecies], dens[kMaxSpecies];
            int np = 0;
            for (int p = 0; p < c->ns; ++p) {
                if (!((S.pm_dir[s] >> p) & 1u)) continue;
                rho[np] = std::sqrt((double)S.cull2[c->chem_h.rmap[s][p]]) / (double)S.h;
                dens[np] = (double)std::max<int64_t>(sp_est[p], 0) / ncell;
                ++np;
            }
            // square boxes in x and y (kx = ky), any depth in z; search_box fixes a cube
            const int klo = c->prm.search_box > 0 ? std::min(c->prm.search_box, kmax) : 1;
            const int khi = c->prm.search_box > 0 ? klo : kmax;
            for (int kx = klo; kx <= khi; ++kx)
                for (int kz = (c->prm.search_box > 0 ? std::min(c->prm.search_box, kzmax) : 1);
                     kz <= (c->prm.search_box > 0 ? std::min(c->prm.search_box, kzmax) : kzmax); ++kz) {
                    const int ky = kx;
                    const double E = per_cell * kx * ky * kz;
                    const double passes = std::max(1.0, std::ceil((E + 2.0 * std::sqrt(E)) / 64.0));
                    double streamed = 0.0;
                    for (int q = 0; q < np; ++q)
                        streamed += dens[q] * (kx + 2.0 * rho[q] + 1.0) * (ky + 2.0 * rho[q] + 1.0) *
                                    std::min((double)nc, kz + 2.0 * rho[q] + 1.0);
                    const double cost = passes * (streamed + 128.0) / std::max(E, 0.5);
                    if (cost < best) {
                        best = cost;
                        best_work = passes * streamed;
                        S.kdim_sp[s] = kx | (ky << 8) | (kz << 16);
                    }
                }
            S.work_sp[s] = (float)best_work;
        }
        // one slice per box for now: assign_splits cuts the long streams once every
        // instance of the step is planned
        int64_t off = 0;
        for (int s = 0; s < c->ns; ++s) {
            S.nsplit_sp[s] = 1;
            S.unit_off_sp[s] = (int32_t)off;
            off += S.pm_dir[s] ? boxes_of(S, s) : 0;
        }
        S.unit_off_sp[c->ns] = (int32_t)off;
    }
    return (int32_t)(nc * nc * nc);
}

// Work units of the species-bin search of one instance.
int64_t units_of(const InstStep& S, int ns) { return S.by_species ? S.unit_off_sp[ns] : 0; }

// Tuning key: occupancy of a grid whose cells equal the largest cutoff, in
// octaves (the second key is kept for the table layout and is always 0).
std::pair<int, int> tune_key(double L, int64_t n_est, double rcmax) {
    const double n = (double)std::max<int64_t>(n_est, 1);
    double ncr = rcmax > 0 ? std::floor(L / (rcmax * kGridMargin)) : 1024.0;
    ncr = std::max(1.0, std::min(ncr, 1024.0));
    const double occ = n / (ncr * ncr * ncr);
    const int ko = std::max(-3, std::min(30, (int)std::floor(std::log2(occ))));
    return {ko, 0};
}

// Process-wide autotuning cache: per key, accumulated step time of every
// configuration tried.  The configuration changes nothing but speed -- the
// candidate set of every step is the same for any grid -- so it is tried on
// live steps of real runs; later runs of the same shape reuse the choice.
struct TuneEntry {
    double ms[kNumCfg] = {};
    int cnt[kNumCfg] = {};
    int pend[kNumCfg] = {};
};
std::mutex g_tune_mu;
std::map<std::pair<int, int>, TuneEntry> g_tune;
constexpr int kTuneSamples = 2;

// species bins only pay off once cutoff-sized cells hold a few molecules
bool cfg_eligible(int cfg, int ko) { return kCfgs[cfg].by_species == 0 || ko >= 0; }

int default_cfg(int ko) { return ko < 3 ? 0 : 4; }

// Configuration for a key: while exploring, the default first and then every
// eligible configuration not yet sampled kTuneSamples times, except those whose
// first sample was more than 3x the best mean so far; else the fastest.
int pick_cfg(std::pair<int, int> key, bool explore_ok, bool* explore) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneEntry& e = g_tune[key];
    if (explore_ok) {
        double best_mean = -1.0;
        for (int k = 0; k < kNumCfg; ++k)
            if (e.cnt[k] > 0 && (best_mean < 0 || e.ms[k] / e.cnt[k] < best_mean)) best_mean = e.ms[k] / e.cnt[k];
        const int d = default_cfg(key.first);
        for (int r = -1; r < kNumCfg; ++r) {
            const int k = r < 0 ? d : r;
            if (r >= 0 && k == d) continue;
            if (!cfg_eligible(k, key.first)) continue;
            if (e.cnt[k] > 0 && best_mean > 0 && e.ms[k] / e.cnt[k] > 3.0 * best_mean) continue;
            if (e.cnt[k] + e.pend[k] < kTuneSamples) {
                if (r >= 0 && e.pend[k] > 0) continue;  // wait for its first sample before a second
                e.pend[k]++;
                if (explore) *explore = true;
                return k;
            }
        }
    }
    int best = -1;
    double bt = 0.0;
    for (int k = 0; k < kNumCfg; ++k) {
        if (!cfg_eligible(k, key.first) || e.cnt[k] == 0) continue;
        const double t = e.ms[k] / e.cnt[k];
        if (best < 0 || t < bt) {
            best = k;
            bt = t;
        }
    }
    return best >= 0 ? best : default_cfg(key.first);
}

void tune_record(std::pair<int, int> key, int cfg, double ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneEntry& e = g_tune[key];
    if (e.pend[cfg] > 0) e.pend[cfg]--;
    e.ms[cfg] += ms;
    e.cnt[cfg]++;
}

StepBuffers buffers(gsbs_ctx* c) {
    StepBuffers b{};
    b.pos_in = c->pos[c->cur];
    b.uid_in = c->uid[c->cur];
    b.pos_out = c->pos[c->cur ^ 1];
    b.uid_out = c->uid[c->cur ^ 1];
    b.pos0_out = c->pos0;
    b.cellrank = c->cellrank;
    b.xnew = c->xnew;
    b.cell_count = c->cell_count;
    b.cell_start = c->cell_start;
    b.scan_status = c->scan_status;
    c->scan_epoch = c->scan_epoch >= 0x7FFFFFFFu ? 1u : c->scan_epoch + 1u;
    b.scan_epoch = c->scan_epoch;
    b.pairs = c->pairs;
    b.pair_cap = c->pair_cap;
    b.claim = c->claim;
    b.mate = c->mate;
    b.counts = c->counts;
    b.msteps = c->msteps;
    b.ctr = c->ctr;
    b.cap = c->cap;
    b.x0_override = c->x0_dbg;
    return b;
}

int run_step(gsbs_ctx* c, const StepBuffers& bf, const InstStep* P, int32_t n_inst, int32_t bins, int32_t units,
             int32_t grid, int32_t flags, hipEvent_t* span = nullptr, const InstStep* row0 = nullptr, int cfg0 = -1,
             int64_t nest0 = 0, hipEvent_t* live = nullptr) {
    if (span) HIPCHK(hipEventRecord(span[0], c->st));
    if (!c->fo.empty()) flags |= kStepFirstOrder;
    if (c->profiling)  // two events per kernel slot (the mask names the six slots, not the chained form)
        launch_step(c->st, bf, P, c->chem_d, n_inst, bins, units, c->ns, grid, flags, c->prof_ev,
                    (1u << kStepKernels) - 1u);
    else
        launch_step(c->st, bf, P, c->chem_d, n_inst, bins, units, c->ns, grid, flags, live, kEvChain);
    HIPCHK(hipGetLastError());
    if (span) HIPCHK(hipEventRecord(span[1], c->st));
    if (c->profiling) {
        HIPCHK(hipEventSynchronize(c->prof_ev[2 * kStepKernels - 1]));
        DevCounters h{};
        HIPCHK(hipMemcpy(&h, c->ctr, sizeof(h), hipMemcpyDeviceToHost));
        const int64_t dcand = (int64_t)(h.cand - c->prof_cand);
        c->prof_cand = h.cand;
        for (int k = 0; k < kStepKernels; ++k) {
            // slots 3 and 4 (whole-cell and species-bin search) run only when some instance uses them
            if ((k == 3 && !(flags & kStepHasWhole)) || (k == 4 && !(flags & kStepHasSpecies))) continue;
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c->prof_ev[2 * k], c->prof_ev[2 * k + 1]));
            c->prof_ms[k] += ms;
            c->prof_n[k] += 1;
        }
        // work units; a step that used both searches counts its molecules and candidates
        // for the species-bin one
        const int ks = (flags & kStepHasSpecies) ? 4 : 3;
        for (int k = 0; k < kStepKernels; ++k)
            if (k != 3 && k != 4) c->prof_work[k] += (k == 1) ? (int64_t)bins : (int64_t)h.n_live;
        c->prof_work[ks] += h.n_live;
        c->prof_cnd[ks] += dcand;
        float tot = 0.f;
        HIPCHK(hipEventElapsedTime(&tot, c->prof_ev[0], c->prof_ev[2 * kStepKernels - 1]));
        if (row0)
            c->step_log.push_back({(int64_t)row0->step, (double)tot, row0->nc, row0->reach, row0->by_species, cfg0,
                                   nest0});
    }
    return GSBS_OK;
}

// Kernel times of a finished chunk of live-timed steps (buffer b).
int live_harvest(gsbs_ctx* c, int b) {
    if (!c->live_pending[b]) return GSBS_OK;
    HIPCHK(hipEventSynchronize(c->live_done[b]));
    for (int k = 0; k < c->live_nstep[b]; ++k) {
        const int32_t fl = c->live_flags[b][k];
        for (int q = 0; q < kStepKernels; ++q) {
            if (!((c->live_mask >> q) & 1u)) continue;
            if ((q == 3 && !(fl & kStepHasWhole)) || (q == 4 && !(fl & kStepHasSpecies))) continue;
            float ms = 0.f;
            const hipEvent_t* e = &c->live_ev[b][(size_t)k * (kStepKernels + 1) + q];
            HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
            c->prof_ms[q] += ms;
            c->prof_n[q] += 1;
        }
    }
    c->live_pending[b] = false;
    c->live_nstep[b] = 0;
    return GSBS_OK;
}

int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    g = std::max<int64_t>(g, 1);
    return (int)std::min<int64_t>(g, 16384);
}

int apply_injection(gsbs_ctx* c, int idx, const Pending& p) {
    InstHost& in = c->inst[idx];
    launch_inject(c->st, c->pos[c->cur], c->uid[c->cur], c->counts, c->ctr, p.d_xyz, p.d_sp, (int32_t)p.n, idx,
                  in.next_uid, c->cap);
    HIPCHK(hipGetLastError());
    in.next_uid += (uint64_t)p.n;
    in.edep += p.edep;
    c->injected[idx] += p.n;
    return GSBS_OK;
}

// Injections due at the instance's present time, then its records there.
int boundary(gsbs_ctx* c, int idx, RecordList& rl) {
    InstHost& in = c->inst[idx];
    std::vector<Pending> keep;
    for (const Pending& p : in.pending) {
        if (p.t <= in.t) {
            CHK(apply_injection(c, idx, p));
            in.n_est += p.n;
            HIPCHK(hipStreamSynchronize(c->st));
            dfree(const_cast<Pending&>(p).d_xyz);
            dfree(const_cast<Pending&>(p).d_sp);
        } else {
            keep.push_back(p);
        }
    }
    in.pending.swap(keep);
    for (size_t r = 0; r < in.rec_t.size(); ++r) {
        if (!in.rec_done[r] && in.rec_t[r] == in.t) {
            in.rec_done[r] = 1;
            in.rec_edep[r] = in.edep;
            if (rl.n == 32) {
                launch_record(c->st, c->counts, c->rec, c->max_rec, rl);
                rl.n = 0;
            }
            rl.inst[rl.n] = idx;
            rl.rec[rl.n] = (int32_t)r;
            rl.n++;
        }
    }
    return GSBS_OK;
}

int check_device_errors(gsbs_ctx* c) {
    DevCounters h{};
    CHK(read_counters(c, &h));
    if (h.err & kErrMolOverflow) return fail(GSBS_ECAPACITY, "molecule capacity exceeded on the device");
    if (h.err & kErrPairOverflow) return fail(GSBS_ECAPACITY, "pair list capacity exceeded on the device");
    if (h.err & kErrTie) return fail(GSBS_ESTATE, "two pairs with identical matching keys");
    if (h.err & kErrScanStall) return fail(GSBS_EHIP, "cell scan: look-back did not complete");
    return GSBS_OK;
}

int refresh_estimates(gsbs_ctx* c) {
    std::vector<long long> cnt((size_t)c->n_inst * kMaxSpecies);
    HIPCHK(hipMemcpyAsync(cnt.data(), c->counts, sizeof(long long) * cnt.size(), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    int64_t tot = 0;
    for (int i = 0; i < c->n_inst; ++i) {
        int64_t s = 0;
        for (int k = 0; k < kMaxSpecies; ++k) {
            s += cnt[(size_t)i * kMaxSpecies + k];
            c->inst[i].sp_est[k] = cnt[(size_t)i * kMaxSpecies + k];
        }
        c->inst[i].n_est = s;
        tot += s;
    }
    c->max_live = std::max<int64_t>(c->max_live, tot);
    return GSBS_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char* gsbs_last_error(void) { return g_err.c_str(); }

int gsbs_default_params(gsbs_params* p) {
    if (!p) return fail(GSBS_EINVAL, "null params");
    p->c_cut = 5.0;
    p->rounds = 4;
    p->contact_only = 0;
    p->dt0_ns = 1e-3;
    p->ratio = std::pow(10.0, 6.0 / 1999.0);
    p->dt_max_ns = 0.0;
    p->grid_config = -1;
    p->autotune = 1;
    p->search_split = 0;
    p->search_box = 0;
    p->step_graph = 0;
    return GSBS_OK;
}

int gsbs_create(const gsbs_box* boxes, int32_t n_instances, uint64_t seed, void* stream, gsbs_ctx** out) {
    if (!boxes || !out || n_instances <= 0 || n_instances > (1 << 23)) return fail(GSBS_EINVAL, "bad instances");
    for (int i = 0; i < n_instances; ++i)
        if (!(boxes[i].L_nm > 0)) return fail(GSBS_EINVAL, "box edge must be positive");
    gsbs_ctx* c = new gsbs_ctx();
    c->n_inst = n_instances;
    c->seed = seed;
    c->st = (hipStream_t)stream;
    gsbs_default_params(&c->prm);
    c->inst.resize(n_instances);
    int64_t cap = 0;
    for (int i = 0; i < n_instances; ++i) {
        c->inst[i].L = boxes[i].L_nm;
        c->inst[i].cap_hint = boxes[i].capacity;
        cap += std::max<int64_t>(boxes[i].capacity, 0);
    }
    int r = GSBS_OK;
    if ((r = dalloc(&c->ctr, 1)) || (r = dalloc(&c->counts, (size_t)n_instances * kMaxSpecies)) ||
        (r = dalloc(&c->msteps, (size_t)n_instances))) {
        gsbs_destroy(c);
        return r;
    }
    hipError_t e = hipMemsetAsync(c->ctr, 0, sizeof(DevCounters), c->st);
    if (e == hipSuccess) e = hipMemsetAsync(c->counts, 0, sizeof(long long) * n_instances * kMaxSpecies, c->st);
    if (e == hipSuccess) e = hipMemsetAsync(c->msteps, 0, sizeof(unsigned long long) * n_instances, c->st);
    c->injected.assign(n_instances, 0);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipHostMalloc((void**)&c->h_cnt[b], sizeof(long long) * kMaxSpecies * n_instances);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->cnt_ev[b], hipEventDisableTiming);
        c->cnt_mark[b].assign(n_instances, 0);
        if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_chunk[b], sizeof(InstStep) * kChunk * n_instances);
        if (e == hipSuccess) e = hipMalloc((void**)&c->d_chunk[b], sizeof(InstStep) * kChunk * n_instances);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->chunk_ev[b], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        gsbs_destroy(c);
        return fail(GSBS_EHIP, std::string("create: ") + hipGetErrorString(e));
    }
    if ((r = ensure_capacity(c, std::max<int64_t>(cap, 4096))) != GSBS_OK || (r = ensure_cells(c, 4096))) {
        gsbs_destroy(c);
        return r;
    }
    *out = c;
    return GSBS_OK;
}

int gsbs_destroy(gsbs_ctx* c) {
    if (!c) return GSBS_OK;
    if (c->st || true) (void)hipStreamSynchronize(c->st);
    for (auto& in : c->inst)
        for (auto& p : in.pending) {
            dfree(p.d_xyz);
            dfree(p.d_sp);
        }
    for (int b = 0; b < 2; ++b) {
        dfree(c->pos[b]);
        dfree(c->uid[b]);
        if (c->h_chunk[b]) (void)hipHostFree(c->h_chunk[b]);
        dfree(c->d_chunk[b]);
        if (c->chunk_ev[b]) (void)hipEventDestroy(c->chunk_ev[b]);
    }
    dfree(c->pos0);
    dfree(c->cellrank);
    dfree(c->claim);
    dfree(c->mate);
    dfree(c->x0_dbg);
    dfree(c->xnew);
    dfree(c->cell_count);
    dfree(c->cell_start);
    dfree(c->scan_status);
    dfree(c->pairs);
    dfree(c->counts);
    dfree(c->msteps);
    dfree(c->ctr);
    dfree(c->rec);
    dfree(c->chem_d);
    for (auto& ge : c->graph_cache) {
        (void)hipGraphExecDestroy(ge.exec);
        (void)hipEventDestroy(ge.done);
    }
    dfree(c->sur_ref_idx);
    dfree(c->sur_ref_cnt);
    dfree(c->sur_pair_ab);
    dfree(c->sur_edges2);
    dfree(c->sur_shell);
    dfree(c->sur_hist);
    dfree(c->sur_vec);
    dfree(c->sur_newc);
    dfree(c->sur_x);
    dfree(c->sur_y);
    for (auto& e : c->prof_ev)
        if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < 2; ++b) {
        for (auto& e : c->live_ev[b])
            if (e) (void)hipEventDestroy(e);
        if (c->live_done[b]) (void)hipEventDestroy(c->live_done[b]);
    }
    for (auto& e : c->tune_ev)
        if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < 2; ++b) {
        if (c->h_cnt[b]) (void)hipHostFree(c->h_cnt[b]);
        if (c->cnt_ev[b]) (void)hipEventDestroy(c->cnt_ev[b]);
    }
    delete c;
    return GSBS_OK;
}

int gsbs_set_species(gsbs_ctx* c, int32_t n, const double* D) {
    if (!c || !D || n <= 0 || n > kMaxSpecies) return fail(GSBS_EINVAL, "species: 1..16 coefficients");
    for (int i = 0; i < n; ++i)
        if (!(D[i] >= 0)) return fail(GSBS_EINVAL, "negative diffusion coefficient");
    c->ns = n;
    c->D.assign(D, D + n);
    c->chem_ready = false;
    if (!c->rx.empty()) return build_chem(c);
    return GSBS_OK;
}

int gsbs_set_reactions(gsbs_ctx* c, int32_t n, const gsbs_reaction* r) {
    if (!c || n < 0 || n > kMaxReactions || (n > 0 && !r)) return fail(GSBS_EINVAL, "reactions: 0..32");
    if (c->ns == 0) return fail(GSBS_ESTATE, "set the species first");
    std::vector<int> seen(kMaxSpecies * kMaxSpecies, 0);
    for (int k = 0; k < n; ++k) {
        const gsbs_reaction& q = r[k];
        if (q.a < 0 || q.b < 0 || q.a >= c->ns || q.b >= c->ns) return fail(GSBS_EINVAL, "reactant species");
        if (q.n_products < 0 || q.n_products > 3) return fail(GSBS_EINVAL, "0..3 products");
        for (int p = 0; p < q.n_products; ++p)
            if (q.products[p] < 0 || q.products[p] >= c->ns) return fail(GSBS_EINVAL, "product species");
        if (!(q.k_in > 0)) return fail(GSBS_EINVAL, "rate constant must be positive");
        if (q.keep_b && (q.a == q.b || q.n_products != 0)) return fail(GSBS_EINVAL, "keep_b needs a != b, no products");
        if (seen[q.a * kMaxSpecies + q.b]++ || (q.a != q.b && seen[q.b * kMaxSpecies + q.a]++))
            return fail(GSBS_EINVAL, "two reactions for one species pair");
    }
    c->rx.assign(r, r + n);
    CHK(build_chem(c));
    for (size_t k = 0; k < c->rx.size(); ++k)
        for (auto& in : c->inst)
            if (2.0 * c->R[k] >= in.L) return fail(GSBS_EMINIMAGE, "2R >= L");
    return GSBS_OK;
}

int gsbs_set_sources(gsbs_ctx* c, int32_t n, const gsbs_source* src) {
    if (!c || n < 0 || n > kMaxSources || (n > 0 && !src)) return fail(GSBS_EINVAL, "sources: 0..4");
    if (c->ns == 0) return fail(GSBS_ESTATE, "set the species first");
    for (int q = 0; q < n; ++q) {
        if (!(src[q].rate_M_per_ns >= 0.0) || !std::isfinite(src[q].rate_M_per_ns))
            return fail(GSBS_EINVAL, "source rate must be finite and >= 0");
        if (src[q].n_products < 1 || src[q].n_products > 3) return fail(GSBS_EINVAL, "1..3 source products");
        for (int k = 0; k < src[q].n_products; ++k)
            if (src[q].products[k] < 0 || src[q].products[k] >= c->ns) return fail(GSBS_EINVAL, "product species");
    }
    c->src.assign(src, src + n);
    return GSBS_OK;
}

int gsbs_set_first_order(gsbs_ctx* c, int32_t n, const gsbs_first_order* f) {
    if (!c || n < 0 || n > kMaxSpecies || (n > 0 && !f)) return fail(GSBS_EINVAL, "first-order channels: 0..16");
    if (c->ns == 0) return fail(GSBS_ESTATE, "set the species first");
    uint32_t seen = 0;
    for (int q = 0; q < n; ++q) {
        if (f[q].a < 0 || f[q].a >= c->ns) return fail(GSBS_EINVAL, "first-order species");
        if ((seen >> f[q].a) & 1u) return fail(GSBS_EINVAL, "one first-order channel per species");
        seen |= 1u << f[q].a;
        if (!(f[q].k_per_ns > 0.0) || !std::isfinite(f[q].k_per_ns))
            return fail(GSBS_EINVAL, "first-order rate must be finite and > 0");
        if (f[q].n_products < 0 || f[q].n_products > 2) return fail(GSBS_EINVAL, "0..2 first-order products");
        for (int k = 0; k < f[q].n_products; ++k)
            if (f[q].products[k] < 0 || f[q].products[k] >= c->ns) return fail(GSBS_EINVAL, "product species");
    }
    c->fo.assign(f, f + n);
    std::sort(c->fo.begin(), c->fo.end(), [](const gsbs_first_order& x, const gsbs_first_order& y) { return x.a < y.a; });
    if (c->chem_ready) CHK(build_chem(c));
    return GSBS_OK;
}

int gsbs_set_params(gsbs_ctx* c, const gsbs_params* p) {
    if (!c || !p) return fail(GSBS_EINVAL, "null");
    if (!(p->c_cut > 0) || p->rounds < 1 || !(p->dt0_ns > 0) || !(p->ratio > 1.0) || p->dt_max_ns < 0 ||
        p->grid_config < -1 || p->grid_config >= kNumCfg || p->search_split < 0 || p->search_split > 16 ||
        p->search_box < 0 || p->search_box > 8 || p->step_graph < 0 || p->step_graph > 1)
        return fail(GSBS_EINVAL, "bad parameters");
    c->prm = *p;
    c->tuning = p->autotune != 0;
    if (c->ns && !c->rx.empty()) return build_chem(c);
    return GSBS_OK;
}

int gsbs_get_radii(gsbs_ctx* c, double* R) {
    if (!c || !R) return fail(GSBS_EINVAL, "null");
    for (size_t k = 0; k < c->R.size(); ++k) R[k] = c->R[k];
    return GSBS_OK;
}

int gsbs_get_dt_max(gsbs_ctx* c, int32_t i, double* dt) {
    if (!c || !dt || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    *dt = c->inst[i].dt_max;
    return GSBS_OK;
}

// Queue an injection (its molecules already in device buffers it owns).
static void queue_pending(InstHost& in, const Pending& p) {
    in.pending.push_back(p);
    std::stable_sort(in.pending.begin(), in.pending.end(), [](const Pending& x, const Pending& y) { return x.t < y.t; });
    in.anchors.push_back(p.t);
    std::sort(in.anchors.begin(), in.anchors.end());
    in.anchors.erase(std::unique(in.anchors.begin(), in.anchors.end()), in.anchors.end());
}

int gsbs_inject(gsbs_ctx* c, int32_t i, double t, int64_t n, const float* xyz, const uint8_t* sp,
                double edep, int32_t device_ptrs) {
    if (!c || i < 0 || i >= c->n_inst || n < 0 || (n > 0 && (!xyz || !sp)))
        return fail(GSBS_EINVAL, "bad injection");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    if (c->ns == 0) return fail(GSBS_ESTATE, "set the species first");
    InstHost& in = c->inst[i];
    if (t < in.t) return fail(GSBS_ESTATE, "injection before the instance's present time");
    if (!device_ptrs) {
        for (int64_t k = 0; k < n; ++k)
            if (sp[k] >= c->ns) return fail(GSBS_EINVAL, "species index out of range");
    }
    int64_t total = 0;
    for (auto& q : c->inst) {
        int64_t pend = 0;
        for (auto& p : q.pending) pend += p.n;
        total += q.n_est + pend;
    }
    total += n;
    // R1-like reactions add one molecule per two consumed: 1.5x covers the worst case
    CHK(ensure_capacity(c, total + total / 2 + 1024));
    Pending p{t, n, nullptr, nullptr, edep};
    if (n > 0) {
        CHK(dalloc(&p.d_xyz, (size_t)n * 3));
        CHK(dalloc(&p.d_sp, (size_t)n));
        const hipMemcpyKind k = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIPCHK(hipMemcpyAsync(p.d_xyz, xyz, sizeof(float) * 3 * n, k, c->st));
        HIPCHK(hipMemcpyAsync(p.d_sp, sp, (size_t)n, k, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    queue_pending(in, p);
    return GSBS_OK;
}

int gsbs_inject_pulse(gsbs_ctx* c, int32_t i, const gsbs_pulse* q, int64_t* n_injected) {
    if (!c || !q || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad pulse");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    if (c->ns == 0) return fail(GSBS_ESTATE, "set the species first");
    InstHost& in = c->inst[i];
    if (!(q->t_ns >= in.t)) return fail(GSBS_ESTATE, "pulse before the instance's present time");
    if (q->n_tracks < 0 || !(q->spacing_nm > 0.0) || !(q->mol_per_spur >= 0.0) || q->mol_per_spur > 30.0 ||
        !(q->sigma_nm >= 0.0) || !(q->let_kev_per_um >= 0.0) || !std::isfinite(q->spacing_nm) ||
        !std::isfinite(q->sigma_nm))
        return fail(GSBS_EINVAL, "bad pulse parameters");
    SpurParams P{};
    double sum = 0.0;
    for (int s = 0; s < c->ns; ++s) {
        if (!(q->frac[s] >= 0.0)) return fail(GSBS_EINVAL, "negative species fraction");
        sum += q->frac[s];
        P.cum[s] = sum;
        if (q->frac[s] > 0.0) P.last = s;
    }
    if (!(std::fabs(sum - 1.0) <= 1e-9)) return fail(GSBS_EINVAL, "species fractions must sum to 1");
    P.L = in.L;
    P.spacing = q->spacing_nm;
    P.mean = q->mol_per_spur;
    P.sigma = q->sigma_nm;
    P.ns = c->ns;
    P.n_tracks = q->n_tracks;
    P.seed = c->seed;
    P.stream = q->stream;
    const int nt = q->n_tracks;
    std::vector<int64_t> cnt((size_t)nt), off((size_t)nt);
    int64_t total = 0;
    int64_t* d_cnt = nullptr;
    float* d_xyz = nullptr;
    uint8_t* d_sp = nullptr;
    struct Release {
        int64_t** a;
        float** x;
        uint8_t** s;
        bool keep = false;
        ~Release() {
            dfree(*a);
            if (!keep) {
                dfree(*x);
                dfree(*s);
            }
        }
    } release{&d_cnt, &d_xyz, &d_sp};
    if (nt > 0) {
        CHK(dalloc(&d_cnt, (size_t)nt));
        launch_spur_count(c->st, P, d_cnt);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int64_t) * nt, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        for (int k = 0; k < nt; ++k) {
            off[(size_t)k] = total;
            total += cnt[(size_t)k];
        }
    }
    if (total > (int64_t)0x7FFFFFF0) return fail(GSBS_ECAPACITY, "pulse beyond 2^31 molecules");
    int64_t pend_all = 0;
    for (auto& qq : c->inst) {
        int64_t pend = 0;
        for (auto& pp : qq.pending) pend += pp.n;
        pend_all += qq.n_est + pend;
    }
    pend_all += total;
    CHK(ensure_capacity(c, pend_all + pend_all / 2 + 1024));
    if (total > 0) {
        CHK(dalloc(&d_xyz, (size_t)total * 3));
        CHK(dalloc(&d_sp, (size_t)total));
        HIPCHK(hipMemcpyAsync(d_cnt, off.data(), sizeof(int64_t) * nt, hipMemcpyHostToDevice, c->st));
        launch_spur_emit(c->st, P, d_cnt, d_xyz, d_sp);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(c->st));
    }
    // deposited energy: tracks of length L at the LET (keV/um x nm = eV)
    Pending p{q->t_ns, total, d_xyz, d_sp, (double)nt * in.L * q->let_kev_per_um};
    release.keep = true;
    queue_pending(in, p);
    if (n_injected) *n_injected = total;
    return GSBS_OK;
}

int gsbs_set_records(gsbs_ctx* c, int32_t i, int32_t n, const double* t) {
    if (!c || i < 0 || i >= c->n_inst || n < 0 || (n > 0 && !t)) return fail(GSBS_EINVAL, "bad records");
    for (int k = 1; k < n; ++k)
        if (!(t[k] > t[k - 1])) return fail(GSBS_EINVAL, "record times must increase");
    if (n > c->max_rec) {
        const int32_t nm = std::max(n, c->max_rec * 2);
        long long* nr = nullptr;
        CHK(dalloc(&nr, (size_t)c->n_inst * nm * kMaxSpecies));
        std::vector<long long> fill((size_t)c->n_inst * nm * kMaxSpecies, -1);
        if (c->rec) {
            std::vector<long long> old((size_t)c->n_inst * c->max_rec * kMaxSpecies);
            HIPCHK(hipMemcpyAsync(old.data(), c->rec, sizeof(long long) * old.size(), hipMemcpyDeviceToHost, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
            for (int q = 0; q < c->n_inst; ++q)
                std::memcpy(&fill[(size_t)q * nm * kMaxSpecies], &old[(size_t)q * c->max_rec * kMaxSpecies],
                            sizeof(long long) * c->max_rec * kMaxSpecies);
        }
        HIPCHK(hipMemcpyAsync(nr, fill.data(), sizeof(long long) * fill.size(), hipMemcpyHostToDevice, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        dfree(c->rec);
        c->rec = nr;
        c->max_rec = nm;
    }
    std::vector<long long> neg((size_t)c->max_rec * kMaxSpecies, -1);
    HIPCHK(hipMemcpyAsync(c->rec + (size_t)i * c->max_rec * kMaxSpecies, neg.data(), sizeof(long long) * neg.size(),
                          hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    InstHost& in = c->inst[i];
    in.rec_t.assign(t, t + n);
    in.rec_done.assign(n, 0);
    in.rec_edep.assign(n, 0.0);
    return GSBS_OK;
}

// Hand-over points of an instance: settle_ns after an injection a_k whose next
// injection a_(k+1) comes later than a_k + settle_ns + min_gap_ns; (time, next).
static void handover_points(const gsbs_ctx* c, const InstHost& in, std::vector<std::pair<double, double>>& out) {
    out.clear();
    if (!c->sur_on) return;
    const double st = c->sur_cfg.settle_ns, gap = c->sur_cfg.min_gap_ns;
    for (size_t k = 0; k + 1 < in.anchors.size(); ++k)
        if (in.anchors[k + 1] - in.anchors[k] > st + gap) out.push_back({in.anchors[k] + st, in.anchors[k + 1]});
}

static int advance_plain(gsbs_ctx* c, const double* target) {
    for (int i = 0; i < c->n_inst; ++i)
        if (target[i] < c->inst[i].t) return fail(GSBS_ESTATE, "target time before the present");
    // schedules
    std::vector<std::vector<double>> sched(c->n_inst);
    size_t G = 0;
    for (int i = 0; i < c->n_inst; ++i) {
        InstHost& in = c->inst[i];
        std::vector<double> ev;
        for (double r : in.rec_t)
            if (r > in.t && r <= target[i]) ev.push_back(r);
        for (auto& p : in.pending)
            if (p.t > in.t && p.t <= target[i]) ev.push_back(p.t);
        // with a surrogate set, hand-over points are step ends in both modes
        std::vector<std::pair<double, double>> hp;
        handover_points(c, in, hp);
        for (auto& q : hp)
            if (q.first > in.t && q.first <= target[i]) ev.push_back(q.first);
        std::sort(ev.begin(), ev.end());
        ev.erase(std::unique(ev.begin(), ev.end()), ev.end());
        plan_steps(in.t, target[i], in.anchors.data(), (int)in.anchors.size(), ev.data(), (int)ev.size(),
                   c->prm.dt0_ns, c->prm.ratio, in.dt_max, sched[i]);
        G = std::max(G, sched[i].size());
    }
    std::vector<double> t0(c->n_inst);
    std::vector<uint64_t> step0(c->n_inst);
    for (int i = 0; i < c->n_inst; ++i) {
        t0[i] = c->inst[i].t;
        step0[i] = c->inst[i].step;
    }
    // boundary at the present time
    RecordList rl{};
    for (int i = 0; i < c->n_inst; ++i) CHK(boundary(c, i, rl));
    launch_record(c->st, c->counts, c->rec, c->max_rec, rl);
    rl.n = 0;

    std::vector<int32_t> total_cells(kChunk);  // bins of the step
    std::vector<int32_t> total_units(kChunk);
    std::vector<int32_t> step_flags(kChunk);
    std::vector<int> tune_cfg(kChunk, -1);
    std::vector<int> step_cfg(kChunk, -1);
    std::vector<int64_t> step_nest(kChunk, 0);
    std::vector<std::pair<int, int>> tune_key_of(kChunk);
    if (c->tuning && !c->tune_ev[0])
        for (auto& e : c->tune_ev) HIPCHK(hipEventCreate(&e));
    for (size_t g0 = 0; g0 < G; g0 += kChunk) {
        const int nstep = (int)std::min<size_t>(kChunk, G - g0);
        const int b = c->chunk_buf;
        HIPCHK(hipEventSynchronize(c->chunk_ev[b]));
        InstStep* hrow = c->h_chunk[b];
        // refresh the live-count estimates from the newest finished copy of the counts
        for (int q = 0; q < 2; ++q) {
            const int sl = (c->cnt_slot + q) & 1;  // older slot first, newer overrides
            if (!c->cnt_pending[sl] || hipEventQuery(c->cnt_ev[sl]) != hipSuccess) continue;
            for (int i = 0; i < c->n_inst; ++i) {
                int64_t s = 0;
                for (int k = 0; k < kMaxSpecies; ++k) {
                    s += c->h_cnt[sl][(size_t)i * kMaxSpecies + k];
                    c->inst[i].sp_est[k] = c->h_cnt[sl][(size_t)i * kMaxSpecies + k];
                }
                c->inst[i].n_est = s + (c->injected[i] - c->cnt_mark[sl][i]);
            }
        }
        // n_est evolves with the injections inside the chunk
        std::vector<int64_t> nest(c->n_inst);
        for (int i = 0; i < c->n_inst; ++i) nest[i] = c->inst[i].n_est;
        int64_t n_total = 0;
        std::vector<double> rcm(c->n_inst);
        for (int k = 0; k < nstep; ++k) {
            const size_t g = g0 + k;
            int lead = -1;
            for (int i = 0; i < c->n_inst; ++i)
                if (g < sched[i].size() && (lead < 0 || nest[i] > nest[lead])) lead = i;
            int32_t base = 0;
            int64_t ubase = 0;
            int32_t fl = 0;
            tune_cfg[k] = -1;
            for (int i = 0; i < c->n_inst; ++i) {
                const bool active = g < sched[i].size();
                const double tprev = (g == 0) ? t0[i] : sched[i][g - 1];
                const double dt = active ? sched[i][g] - tprev : 0.0;
                const uint64_t stp = step0[i] + (uint64_t)std::min<size_t>(g, sched[i].size());
                InstStep& row = hrow[(size_t)k * c->n_inst + i];
                rcm[i] = fill_physics(c, c->inst[i].L, stp, i, dt, active, row);
                int cfg;
                if (c->prm.grid_config >= 0) {
                    cfg = c->prm.grid_config;
                } else {
                    const auto key = tune_key(c->inst[i].L, nest[i], rcm[i]);
                    bool explore = false;
                    cfg = pick_cfg(key, i == lead && c->tuning, &explore);
                    if (explore) {
                        tune_cfg[k] = cfg;
                        tune_key_of[k] = key;
                    }
                }
                row.bin_base = base;
                if (i == 0) {
                    step_cfg[k] = cfg;
                    step_nest[k] = nest[i];
                }
                const int32_t cells = fill_grid(c, c->inst[i].sp_est, c->inst[i].L, nest[i], rcm[i], kCfgs[cfg], 0, row);
                base += row.by_species ? cells * c->ns : cells;
                if (active) fl |= row.by_species ? kStepHasSpecies : kStepHasWhole;
                if (active)
                    for (auto& p : c->inst[i].pending)
                        if (p.t == sched[i][g]) nest[i] += p.n;
            }
            assign_splits(c, &hrow[(size_t)k * c->n_inst], c->n_inst);
            for (int i = 0; i < c->n_inst; ++i) {
                InstStep& row = hrow[(size_t)k * c->n_inst + i];
                row.unit_base = (int32_t)std::min<int64_t>(ubase, 0x7FFFFFF0);
                ubase += units_of(row, c->ns);
            }
            total_cells[k] = base;
            total_units[k] = (int32_t)std::min<int64_t>(ubase, 0x7FFFFFF0);
            step_flags[k] = fl;
        }
        for (int i = 0; i < c->n_inst; ++i) n_total += std::max(nest[i], c->inst[i].n_est);
        int64_t maxc = 0;
        for (int k = 0; k < nstep; ++k) maxc = std::max<int64_t>(maxc, (int64_t)total_cells[k]);
        if (maxc > 0x7FFFFFF0) return fail(GSBS_ECAPACITY, "search grid too large");
        CHK(ensure_cells(c, maxc));
        HIPCHK(hipMemcpyAsync(c->d_chunk[b], hrow, sizeof(InstStep) * nstep * c->n_inst, hipMemcpyHostToDevice,
                              c->st));
        HIPCHK(hipEventRecord(c->chunk_ev[b], c->st));
        c->chunk_buf ^= 1;
        // HIP graph of the chunk's launches, cut before every injection (which synchronises)
        bool explore_chunk = false;
        for (int k = 0; k < nstep; ++k) explore_chunk = explore_chunk || tune_cfg[k] >= 0;
        // (the legacy null stream cannot be captured)
        const bool live = c->live_mask != 0 && !c->profiling;
        const bool use_graph = c->prm.step_graph && !c->profiling && !live && !explore_chunk && c->st != nullptr;
        if (live) {
            CHK(live_harvest(c, b));
            c->live_nstep[b] = nstep;
            for (int k = 0; k < nstep; ++k) c->live_flags[b][k] = step_flags[k];
        }
        bool capturing = false;
        auto flush_graph = [&]() -> int {
            if (!capturing) return GSBS_OK;
            capturing = false;
            hipGraph_t gr = nullptr;
            HIPCHK(hipStreamEndCapture(c->st, &gr));
            // reuse an idle cached executable graph of the same shape, else
            // instantiate one and keep it (two of one shape then alternate)
            gsbs_ctx::GraphEntry* use = nullptr;
            for (auto& ge : c->graph_cache) {
                if (hipEventQuery(ge.done) != hipSuccess) continue;  // still running: leave it
                hipGraphNode_t err_node = nullptr;
                hipGraphExecUpdateResult res{};
                if (hipGraphExecUpdate(ge.exec, gr, &err_node, &res) == hipSuccess) {
                    use = &ge;
                    c->graph_updated++;
                    break;
                }
                (void)hipGetLastError();  // a failed update leaves an error to clear
            }
            if (!use) {
                hipGraphExec_t ex = nullptr;
                const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                if (ei != hipSuccess) {
                    (void)hipGraphDestroy(gr);
                    return fail(GSBS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
                }
                hipEvent_t ev = nullptr;
                HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
                if (c->graph_cache.size() >= 8) {  // keep the most recently used shapes
                    auto old = std::min_element(c->graph_cache.begin(), c->graph_cache.end(),
                                                [](const gsbs_ctx::GraphEntry& a, const gsbs_ctx::GraphEntry& b) { return a.uses < b.uses; });
                    HIPCHK(hipEventSynchronize(old->done));
                    (void)hipGraphExecDestroy(old->exec);
                    (void)hipEventDestroy(old->done);
                    c->graph_cache.erase(old);
                }
                c->graph_cache.push_back({ex, ev, 0});
                use = &c->graph_cache.back();
                c->graph_instantiated++;
            }
            (void)hipGraphDestroy(gr);
            use->uses = (uint64_t)c->steps;
            HIPCHK(hipGraphLaunch(use->exec, c->st));
            HIPCHK(hipEventRecord(use->done, c->st));
            return GSBS_OK;
        };
        for (int k = 0; k < nstep; ++k) {
            const size_t g = g0 + k;
            if (use_graph && !capturing) {
                HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeRelaxed));
                capturing = true;
            }
            StepBuffers bf = buffers(c);
            CHK(run_step(c, bf, c->d_chunk[b] + (size_t)k * c->n_inst, c->n_inst, total_cells[k], total_units[k],
                         grid_for(n_total),
                         step_flags[k], tune_cfg[k] >= 0 ? &c->tune_ev[2 * k] : nullptr,
                         &hrow[(size_t)k * c->n_inst], step_cfg[k], step_nest[k],
                         live ? &c->live_ev[b][(size_t)k * (kStepKernels + 1)] : nullptr));
            if (live) c->live_bins += total_cells[k];
            c->cur ^= 1;
            c->steps++;
            for (int i = 0; i < c->n_inst; ++i) {
                if (g >= sched[i].size()) continue;
                c->inst[i].t = sched[i][g];
                c->inst[i].step++;
                bool due = false;
                for (const Pending& p : c->inst[i].pending) due = due || p.t <= c->inst[i].t;
                if (due) CHK(flush_graph());
                CHK(boundary(c, i, rl));
            }
            if (rl.n) {
                launch_record(c->st, c->counts, c->rec, c->max_rec, rl);
                rl.n = 0;
            }
        }
        CHK(flush_graph());
        if (live) {
            HIPCHK(hipEventRecord(c->live_done[b], c->st));
            c->live_pending[b] = true;
        }
        for (int i = 0; i < c->n_inst; ++i) c->inst[i].n_est = nest[i];
        {
            const int sl = c->cnt_slot;
            if (!c->cnt_pending[sl] || hipEventQuery(c->cnt_ev[sl]) == hipSuccess) {
                HIPCHK(hipMemcpyAsync(c->h_cnt[sl], c->counts, sizeof(long long) * kMaxSpecies * c->n_inst,
                                      hipMemcpyDeviceToHost, c->st));
                HIPCHK(hipEventRecord(c->cnt_ev[sl], c->st));
                c->cnt_pending[sl] = true;
                c->cnt_mark[sl] = c->injected;
                c->cnt_slot ^= 1;
            }
        }
        bool any = false;
        for (int k = 0; k < nstep; ++k) any = any || tune_cfg[k] >= 0;
        if (any) {
            HIPCHK(hipStreamSynchronize(c->st));
            for (int k = 0; k < nstep; ++k) {
                if (tune_cfg[k] < 0) continue;
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, c->tune_ev[2 * k], c->tune_ev[2 * k + 1]));
                tune_record(tune_key_of[k], tune_cfg[k], ms);
            }
        }
    }
    for (int i = 0; i < c->n_inst; ++i) c->inst[i].t = target[i];
    HIPCHK(hipStreamSynchronize(c->st));
    for (int b = 0; b < 2; ++b) CHK(live_harvest(c, b));

    CHK(check_device_errors(c));
    return refresh_estimates(c);
}

int gsbs_advance_to(gsbs_ctx* c, const double* target, int32_t mode) {
    if (!c || !target) return fail(GSBS_EINVAL, "null");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    if (mode != GSBS_PLAIN && mode != GSBS_SURROGATE) return fail(GSBS_EINVAL, "mode: GSBS_PLAIN or GSBS_SURROGATE");
    for (int i = 0; i < c->n_inst; ++i)
        if (!(target[i] >= c->inst[i].t)) return fail(GSBS_ESTATE, "target time before the present");
    if (mode == GSBS_PLAIN) return advance_plain(c, target);
    if (!c->sur_on) return fail(GSBS_ESTATE, "GSBS_SURROGATE without a surrogate (gsbs_set_surrogate)");
    const gsbs_surrogate& q = c->sur_cfg;
    std::vector<double> stop((size_t)c->n_inst), next((size_t)c->n_inst);
    std::vector<std::pair<double, double>> hp;
    std::vector<int> at;
    std::vector<float> xrow((size_t)c->n_inst * kFeatures);
    for (;;) {
        // every instance runs to its next hand-over point not handled yet, else to its target
        at.clear();
        for (int i = 0; i < c->n_inst; ++i) {
            InstHost& in = c->inst[(size_t)i];
            stop[(size_t)i] = target[i];
            handover_points(c, in, hp);
            for (auto& h : hp)
                if (h.first >= in.t && h.first > in.sur_done && h.second <= target[i]) {
                    stop[(size_t)i] = h.first;
                    next[(size_t)i] = h.second;
                    at.push_back(i);
                    break;
                }
        }
        CHK(advance_plain(c, stop.data()));
        if (at.empty()) return GSBS_OK;
        // features of the instances at their hand-over point, one row each, then the network
        for (size_t k = 0; k < at.size(); ++k) {
            const int i = at[k];
            CHK(gsbs_features(c, i, next[(size_t)i] - stop[(size_t)i], q.r_max_nm, q.n_ref_max, q.c_floor_M,
                              c->sur_mu.data(), c->sur_sd.data(), c->sur_x + k * kFeatures, 1));
        }
        HIPCHK(hipMemcpy(xrow.data(), c->sur_x, sizeof(float) * kFeatures * at.size(), hipMemcpyDeviceToHost));
        CHK(mlp_forward_sync(c->sur_net, c->sur_x, (int)at.size(), c->sur_y));
        for (size_t k = 0; k < at.size(); ++k) {
            const int i = at[k];
            InstHost& in = c->inst[(size_t)i];
            const double t_sw = stop[(size_t)i], t_nx = next[(size_t)i];
            // table entry of the interval's bin; +inf outside the edges or the inputs' range
            double est = INFINITY;
            std::vector<int64_t> cnt((size_t)c->ns);
            CHK(gsbs_get_current_counts(c, i, cnt.data()));
            double n_tot = 0;
            for (int64_t v : cnt) n_tot += (double)v;
            const double c_tot = n_tot / (6.02214076e23 * in.L * in.L * in.L * 1e-24);
            const double ldt = std::log10(t_nx - t_sw), lc = std::log10(c_tot);
            const auto& de = c->sur_dt_edges;
            const auto& ce = c->sur_c_edges;
            if (ldt >= de.front() && ldt <= de.back() && c_tot > 0 && lc >= ce.front() && lc <= ce.back()) {
                int a = (int)(std::upper_bound(de.begin(), de.end(), ldt) - de.begin()) - 1;
                int b = (int)(std::upper_bound(ce.begin(), ce.end(), lc) - ce.begin()) - 1;
                a = std::min(std::max(a, 0), q.n_dt - 1);
                b = std::min(std::max(b, 0), q.n_c - 1);
                est = c->sur_table[(size_t)a * q.n_c + b];
            }
            if (!c->sur_lo.empty()) {
                const float* x = &xrow[k * kFeatures];
                for (int f = 0; f < kFeatures; ++f) {
                    const double span = (double)c->sur_hi[f] - (double)c->sur_lo[f];
                    const double m = q.guard_margin * span + 1e-3;
                    if (!((double)x[f] >= (double)c->sur_lo[f] - m && (double)x[f] <= (double)c->sur_hi[f] + m))
                        est = INFINITY;
                }
            }
            const bool take = est <= q.tol && (q.budget <= 0 || in.sur_spent + est <= q.budget);
            in.sur_done = t_sw;
            in.sur_log.push_back({t_sw, t_nx, est, take ? 1 : 0});
            if (take) {
                in.sur_spent += est;
                CHK(gsbs_repopulate(c, i, t_nx, c->sur_y + k * kMlpOut, 1, c->sur_mu_y.data(), c->sur_sd_y.data(),
                                    q.c_floor_M, 1));
            }
        }
    }
}

int gsbs_set_surrogate(gsbs_ctx* c, gsbs_mlp* net, const gsbs_surrogate* q) {
    if (!c) return fail(GSBS_EINVAL, "null");
    for (auto& in : c->inst) {
        in.sur_spent = 0;
        in.sur_done = -INFINITY;
        in.sur_log.clear();
    }
    if (!net && !q) {
        c->sur_on = false;
        c->sur_net = nullptr;
        return GSBS_OK;
    }
    if (!net || !q || !q->mu || !q->sd || !q->mu_y || !q->sd_y || !q->dt_edges || !q->c_edges || !q->table ||
        (!q->lo) != (!q->hi))
        return fail(GSBS_EINVAL, "surrogate: network, normalisation, edges and table are required");
    if (q->n_dt < 1 || q->n_dt > 16 || q->n_c < 1 || q->n_c > 16 || !(q->settle_ns > 0) || !(q->min_gap_ns >= 0) ||
        !(q->tol >= 0) || !(q->guard_margin >= 0) || !(q->r_max_nm > 0) || !(q->c_floor_M > 0) || q->n_ref_max < 1 ||
        !std::isfinite(q->settle_ns) || !std::isfinite(q->budget))
        return fail(GSBS_EINVAL, "surrogate: bad parameters");
    if (!c->chem_ready || c->ns != 7 || c->rx.size() != 9)
        return fail(GSBS_ESTATE, "surrogate: features are defined for 7 species and 9 reactions");
    for (int f = 0; f < kFeatures; ++f)
        if (!(q->sd[f] > 0) || !std::isfinite(q->mu[f])) return fail(GSBS_EINVAL, "surrogate: feature scales");
    for (int k = 0; k < kMlpOut; ++k)
        if (!(q->sd_y[k] > 0) || !std::isfinite(q->mu_y[k])) return fail(GSBS_EINVAL, "surrogate: output scales");
    for (int k = 0; k < q->n_dt; ++k)
        if (!(q->dt_edges[k + 1] > q->dt_edges[k])) return fail(GSBS_EINVAL, "surrogate: dt edges must ascend");
    for (int k = 0; k < q->n_c; ++k)
        if (!(q->c_edges[k + 1] > q->c_edges[k])) return fail(GSBS_EINVAL, "surrogate: concentration edges must ascend");
    if (!c->sur_x) {
        CHK(dalloc(&c->sur_x, (size_t)c->n_inst * kFeatures));
        CHK(dalloc(&c->sur_y, (size_t)c->n_inst * kMlpOut));
    }
    c->sur_cfg = *q;
    c->sur_mu.assign(q->mu, q->mu + kFeatures);
    c->sur_sd.assign(q->sd, q->sd + kFeatures);
    c->sur_lo.clear();
    c->sur_hi.clear();
    if (q->lo) {
        c->sur_lo.assign(q->lo, q->lo + kFeatures);
        c->sur_hi.assign(q->hi, q->hi + kFeatures);
    }
    c->sur_mu_y.assign(q->mu_y, q->mu_y + kMlpOut);
    c->sur_sd_y.assign(q->sd_y, q->sd_y + kMlpOut);
    c->sur_dt_edges.assign(q->dt_edges, q->dt_edges + q->n_dt + 1);
    c->sur_c_edges.assign(q->c_edges, q->c_edges + q->n_c + 1);
    c->sur_table.assign(q->table, q->table + (size_t)q->n_dt * q->n_c);
    c->sur_cfg.mu = c->sur_cfg.sd = c->sur_cfg.lo = c->sur_cfg.hi = c->sur_cfg.mu_y = c->sur_cfg.sd_y = nullptr;
    c->sur_cfg.dt_edges = c->sur_cfg.c_edges = c->sur_cfg.table = nullptr;
    c->sur_net = net;
    c->sur_on = true;
    return GSBS_OK;
}

int gsbs_get_handover_log(gsbs_ctx* c, int32_t i, int64_t max_n, double* t_switch, double* t_next, double* estimate,
                          int32_t* taken, int64_t* n) {
    if (!c || !n || i < 0 || i >= c->n_inst || max_n < 0) return fail(GSBS_EINVAL, "bad arguments");
    const auto& lg = c->inst[(size_t)i].sur_log;
    for (int64_t k = 0; k < std::min<int64_t>(max_n, (int64_t)lg.size()); ++k) {
        if (t_switch) t_switch[k] = lg[(size_t)k].t_switch;
        if (t_next) t_next[k] = lg[(size_t)k].t_next;
        if (estimate) estimate[k] = lg[(size_t)k].estimate;
        if (taken) taken[k] = lg[(size_t)k].taken;
    }
    *n = (int64_t)lg.size();
    return GSBS_OK;
}

int gsbs_sync(gsbs_ctx* c) {
    if (!c) return fail(GSBS_EINVAL, "null");
    HIPCHK(hipStreamSynchronize(c->st));
    return GSBS_OK;
}

// ------------------------------------------------------------ checkpoint ---
extern "C++" {
namespace {

constexpr uint64_t kCkptMagic = 0x31504b4353425347ull;  // "GSBSCKP1"

struct Writer {
    std::vector<char> b;
    template <typename T>
    void put(const T& v) {
        const char* p = reinterpret_cast<const char*>(&v);
        b.insert(b.end(), p, p + sizeof(T));
    }
    void raw(const void* p, size_t n) {
        const char* q = static_cast<const char*>(p);
        b.insert(b.end(), q, q + n);
    }
    template <typename T>
    void vec(const std::vector<T>& v) {
        put<uint64_t>(v.size());
        if (!v.empty()) raw(v.data(), sizeof(T) * v.size());
    }
};

struct Reader {
    const char* p;
    size_t n, at = 0;
    bool ok = true;
    template <typename T>
    T get() {
        T v{};
        if (at + sizeof(T) > n) {
            ok = false;
            return v;
        }
        std::memcpy(&v, p + at, sizeof(T));
        at += sizeof(T);
        return v;
    }
    void raw(void* q, size_t m) {
        if (at + m > n) {
            ok = false;
            return;
        }
        std::memcpy(q, p + at, m);
        at += m;
    }
    template <typename T>
    std::vector<T> vec(size_t limit) {
        const uint64_t m = get<uint64_t>();
        std::vector<T> v;
        if (!ok || m > limit || at + sizeof(T) * m > n) {
            ok = false;
            return v;
        }
        v.resize((size_t)m);
        raw(v.data(), sizeof(T) * m);
        return v;
    }
};

}  // namespace
}  // extern "C++"

int gsbs_save(gsbs_ctx* c, void* buf, int64_t cap, int64_t* size) {
    if (!c || !size || cap < 0 || (cap > 0 && !buf)) return fail(GSBS_EINVAL, "bad checkpoint arguments");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    HIPCHK(hipStreamSynchronize(c->st));
    Writer w;
    w.put(kCkptMagic);
    w.put<int32_t>(c->n_inst);
    w.put<uint64_t>(c->seed);
    w.put(c->prm);
    w.vec(c->D);
    w.vec(c->rx);
    w.vec(c->src);
    w.vec(c->fo);
    w.put<int64_t>(c->steps);
    w.put<int64_t>(c->max_live);
    w.vec(c->injected);
    for (const InstHost& in : c->inst) {
        w.put(in.L);
        w.put(in.cap_hint);
        w.put(in.t);
        w.put(in.step);
        w.put(in.next_uid);
        w.put(in.edep);
        w.put(in.n_est);
        w.raw(in.sp_est, sizeof(in.sp_est));
        w.put(in.dt_max);
        w.vec(in.anchors);
        w.vec(in.rec_t);
        w.vec(in.rec_done);
        w.vec(in.rec_edep);
        w.put<uint64_t>(in.pending.size());
        for (const Pending& q : in.pending) {
            w.put(q.t);
            w.put(q.n);
            w.put(q.edep);
            std::vector<float> xyz((size_t)q.n * 3);
            std::vector<uint8_t> sp((size_t)q.n);
            if (q.n > 0) {
                HIPCHK(hipMemcpy(xyz.data(), q.d_xyz, sizeof(float) * xyz.size(), hipMemcpyDeviceToHost));
                HIPCHK(hipMemcpy(sp.data(), q.d_sp, sp.size(), hipMemcpyDeviceToHost));
            }
            w.raw(xyz.data(), sizeof(float) * xyz.size());
            w.raw(sp.data(), sp.size());
        }
    }
    DevCounters h{};
    HIPCHK(hipMemcpy(&h, c->ctr, sizeof(h), hipMemcpyDeviceToHost));
    w.put(h);
    const int32_t nin = h.n_in;
    std::vector<float4> pos((size_t)std::max(nin, 0));
    std::vector<uint64_t> uid((size_t)std::max(nin, 0));
    if (nin > 0) {
        HIPCHK(hipMemcpy(pos.data(), c->pos[c->cur], sizeof(float4) * nin, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(uid.data(), c->uid[c->cur], sizeof(uint64_t) * nin, hipMemcpyDeviceToHost));
    }
    w.vec(pos);
    w.vec(uid);
    std::vector<long long> cnt((size_t)c->n_inst * kMaxSpecies);
    std::vector<unsigned long long> ms((size_t)c->n_inst);
    HIPCHK(hipMemcpy(cnt.data(), c->counts, sizeof(long long) * cnt.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ms.data(), c->msteps, sizeof(unsigned long long) * ms.size(), hipMemcpyDeviceToHost));
    w.vec(cnt);
    w.vec(ms);
    std::vector<long long> rec((size_t)c->n_inst * c->max_rec * kMaxSpecies);
    if (!rec.empty())
        HIPCHK(hipMemcpy(rec.data(), c->rec, sizeof(long long) * rec.size(), hipMemcpyDeviceToHost));
    w.put<int32_t>(c->max_rec);
    w.vec(rec);
    *size = (int64_t)w.b.size();
    if (!buf) return GSBS_OK;
    if (cap < *size) return fail(GSBS_ECAPACITY, "checkpoint buffer too small");
    std::memcpy(buf, w.b.data(), w.b.size());
    return GSBS_OK;
}

// Molecule record of a checkpoint: finite position inside its cube, instance
// field below n_inst, species below ns (or the removed flag).
static bool valid_record(const float4& p, const std::vector<InstHost>& inst, int ns, int* out_inst, int* out_sp) {
    int meta;
    std::memcpy(&meta, &p.w, 4);
    const int q = meta >> 8, sp = meta & 0xFF;
    if (q < 0 || q >= (int)inst.size() || (sp >= ns && sp != kDead)) return false;
    const float hL = 0.5f * (float)inst[(size_t)q].L;
    for (float x : {p.x, p.y, p.z})
        if (!(x >= -hL && x < hL)) return false;
    *out_inst = q;
    *out_sp = sp;
    return true;
}

int gsbs_load(gsbs_ctx* c, const void* buf, int64_t size) {
    if (!c || !buf || size <= 0) return fail(GSBS_EINVAL, "bad checkpoint arguments");
    Reader r{static_cast<const char*>(buf), (size_t)size};
    if (r.get<uint64_t>() != kCkptMagic || !r.ok) return fail(GSBS_EINVAL, "not a checkpoint");
    if (r.get<int32_t>() != c->n_inst) return fail(GSBS_EINVAL, "checkpoint of another number of instances");
    // 1. parse and check everything on the host; the context is not touched
    const uint64_t seed = r.get<uint64_t>();
    const gsbs_params prm = r.get<gsbs_params>();
    const std::vector<double> D = r.vec<double>(kMaxSpecies);
    const std::vector<gsbs_reaction> rx = r.vec<gsbs_reaction>(kMaxReactions);
    const std::vector<gsbs_source> src = r.vec<gsbs_source>(kMaxSources);
    const std::vector<gsbs_first_order> fo = r.vec<gsbs_first_order>(kMaxSpecies);
    const int64_t steps = r.get<int64_t>(), max_live = r.get<int64_t>();
    const std::vector<int64_t> injected = r.vec<int64_t>((size_t)c->n_inst);
    if (!r.ok || D.empty() || injected.size() != (size_t)c->n_inst) return fail(GSBS_EINVAL, "truncated checkpoint");
    const int ns = (int)D.size();
    std::vector<InstHost> inst((size_t)c->n_inst);
    struct PendingHost {
        double t, edep;
        int64_t n;
        std::vector<float> xyz;
        std::vector<uint8_t> sp;
    };
    std::vector<std::vector<PendingHost>> pend((size_t)c->n_inst);
    for (int i = 0; i < c->n_inst; ++i) {
        InstHost& in = inst[(size_t)i];
        in.L = r.get<double>();
        in.cap_hint = r.get<int64_t>();
        in.t = r.get<double>();
        in.step = r.get<uint64_t>();
        in.next_uid = r.get<uint64_t>();
        in.edep = r.get<double>();
        in.n_est = r.get<int64_t>();
        r.raw(in.sp_est, sizeof(in.sp_est));
        in.dt_max = r.get<double>();
        in.anchors = r.vec<double>(1u << 30);
        in.rec_t = r.vec<double>(1u << 30);
        in.rec_done = r.vec<char>(1u << 30);
        in.rec_edep = r.vec<double>(1u << 30);
        const uint64_t np = r.get<uint64_t>();
        if (!r.ok || np > (1u << 24)) return fail(GSBS_EINVAL, "truncated checkpoint");
        if (in.L != c->inst[(size_t)i].L) return fail(GSBS_EINVAL, "checkpoint of another box");
        if (!std::isfinite(in.t) || in.t < 0 || !std::isfinite(in.edep) || in.rec_done.size() != in.rec_t.size() ||
            in.rec_edep.size() != in.rec_t.size() || !std::is_sorted(in.anchors.begin(), in.anchors.end()))
            return fail(GSBS_EINVAL, "inconsistent instance in the checkpoint");
        for (size_t k = 1; k < in.rec_t.size(); ++k)
            if (!(in.rec_t[k] > in.rec_t[k - 1])) return fail(GSBS_EINVAL, "record times must increase");
        const float hL = 0.5f * (float)in.L;
        for (uint64_t k = 0; k < np && r.ok; ++k) {
            PendingHost q;
            q.t = r.get<double>();
            q.n = r.get<int64_t>();
            q.edep = r.get<double>();
            if (!r.ok || q.n < 0 || (size_t)q.n > r.n) return fail(GSBS_EINVAL, "truncated checkpoint");
            if (!(q.t >= in.t) || !std::isfinite(q.t)) return fail(GSBS_EINVAL, "queued injection before the present");
            q.xyz.resize((size_t)q.n * 3);
            q.sp.resize((size_t)q.n);
            r.raw(q.xyz.data(), sizeof(float) * q.xyz.size());
            r.raw(q.sp.data(), q.sp.size());
            for (int64_t m = 0; m < q.n && r.ok; ++m) {
                if (q.sp[(size_t)m] >= ns) return fail(GSBS_EINVAL, "queued molecule of an unknown species");
                for (int a = 0; a < 3; ++a) {
                    const float x = q.xyz[(size_t)m * 3 + a];
                    if (!(x >= -hL && x < hL)) return fail(GSBS_EINVAL, "queued molecule outside its cube");
                }
            }
            pend[(size_t)i].push_back(std::move(q));
        }
    }
    const DevCounters h = r.get<DevCounters>();
    const std::vector<float4> pos = r.vec<float4>(1u << 31);
    const std::vector<uint64_t> uid = r.vec<uint64_t>(1u << 31);
    const std::vector<long long> cnt = r.vec<long long>((size_t)c->n_inst * kMaxSpecies);
    const std::vector<unsigned long long> ms = r.vec<unsigned long long>((size_t)c->n_inst);
    const int32_t max_rec = r.get<int32_t>();
    const std::vector<long long> rec = r.vec<long long>(1u << 30);
    if (!r.ok || r.at != r.n || pos.size() != uid.size() || (int64_t)pos.size() != (int64_t)h.n_in ||
        cnt.size() != (size_t)c->n_inst * kMaxSpecies || ms.size() != (size_t)c->n_inst || max_rec < 0 ||
        rec.size() != (size_t)c->n_inst * (size_t)max_rec * kMaxSpecies)
        return fail(GSBS_EINVAL, "inconsistent checkpoint");
    if (h.err != 0 || h.n_live < 0 || h.n_live > h.n_in) return fail(GSBS_EINVAL, "checkpoint of a failed context");
    // every record holds a known species of a known instance inside its cube, and
    // the species counts are those of the live records
    std::vector<long long> tally((size_t)c->n_inst * kMaxSpecies, 0);
    for (const float4& p : pos) {
        int q = 0, sp = 0;
        if (!valid_record(p, inst, ns, &q, &sp)) return fail(GSBS_EINVAL, "checkpoint record out of range");
        if (sp != kDead) tally[(size_t)q * kMaxSpecies + sp]++;
    }
    if (tally != cnt) return fail(GSBS_EINVAL, "checkpoint counts differ from its molecules");
    for (size_t i = 0; i < (size_t)c->n_inst; ++i)
        for (size_t k = 0; k < inst[i].rec_t.size() && k < (size_t)max_rec; ++k)
            for (int sp = 0; sp < kMaxSpecies; ++sp)
                if (rec[(i * (size_t)max_rec + k) * kMaxSpecies + sp] < -1)
                    return fail(GSBS_EINVAL, "checkpoint records out of range");
    // 2. device buffers of the new state, before anything of the old one is freed
    int64_t need = (int64_t)pos.size();
    for (int i = 0; i < c->n_inst; ++i)
        for (const PendingHost& q : pend[(size_t)i]) need += q.n;
    std::vector<std::vector<Pending>> npend((size_t)c->n_inst);
    long long* nrec = nullptr;
    auto release_new = [&]() {
        for (auto& v : npend)
            for (auto& p : v) {
                dfree(p.d_xyz);
                dfree(p.d_sp);
            }
        dfree(nrec);
    };
    int rc = GSBS_OK;
    for (int i = 0; i < c->n_inst && rc == GSBS_OK; ++i)
        for (const PendingHost& q : pend[(size_t)i]) {
            Pending p{q.t, q.n, nullptr, nullptr, q.edep};
            if (q.n > 0 && ((rc = dalloc(&p.d_xyz, (size_t)q.n * 3)) != GSBS_OK ||
                            (rc = dalloc(&p.d_sp, (size_t)q.n)) != GSBS_OK)) {
                npend[(size_t)i].push_back(p);
                break;
            }
            npend[(size_t)i].push_back(p);
        }
    if (rc == GSBS_OK && max_rec > c->max_rec) rc = dalloc(&nrec, rec.size());
    if (rc == GSBS_OK) rc = ensure_capacity(c, need + need / 2 + 1024);  // keeps the old molecules if it fails
    if (rc != GSBS_OK) {
        release_new();
        return rc;
    }
    // 3. apply; a failure from here on leaves the context unusable until a load succeeds
    c->broken = true;
    CHK(gsbs_set_species(c, (int32_t)D.size(), D.data()));
    CHK(gsbs_set_params(c, &prm));
    CHK(gsbs_set_reactions(c, (int32_t)rx.size(), rx.data()));
    CHK(gsbs_set_sources(c, (int32_t)src.size(), src.data()));
    CHK(gsbs_set_first_order(c, (int32_t)fo.size(), fo.data()));
    c->seed = seed;
    HIPCHK(hipStreamSynchronize(c->st));
    for (int i = 0; i < c->n_inst; ++i) {
        for (size_t k = 0; k < pend[(size_t)i].size(); ++k) {
            const PendingHost& q = pend[(size_t)i][k];
            const Pending& p = npend[(size_t)i][k];
            if (q.n > 0) {
                HIPCHK(hipMemcpy(p.d_xyz, q.xyz.data(), sizeof(float) * q.xyz.size(), hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(p.d_sp, q.sp.data(), q.sp.size(), hipMemcpyHostToDevice));
            }
        }
    }
    for (auto& in : c->inst)
        for (auto& q : in.pending) {
            dfree(q.d_xyz);
            dfree(q.d_sp);
        }
    for (int i = 0; i < c->n_inst; ++i) {
        InstHost& in = c->inst[(size_t)i];
        in = inst[(size_t)i];
        in.pending = npend[(size_t)i];
    }
    if (nrec) {
        dfree(c->rec);
        c->rec = nrec;
    }
    c->max_rec = max_rec;
    if (!rec.empty()) HIPCHK(hipMemcpy(c->rec, rec.data(), sizeof(long long) * rec.size(), hipMemcpyHostToDevice));
    if (!pos.empty()) {
        HIPCHK(hipMemcpy(c->pos[c->cur], pos.data(), sizeof(float4) * pos.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->uid[c->cur], uid.data(), sizeof(uint64_t) * uid.size(), hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(c->ctr, &h, sizeof(h), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->counts, cnt.data(), sizeof(long long) * cnt.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->msteps, ms.data(), sizeof(unsigned long long) * ms.size(), hipMemcpyHostToDevice));
    c->steps = steps;
    c->max_live = max_live;
    c->injected = injected;
    c->broken = false;
    return GSBS_OK;
}

int gsbs_get_counts(gsbs_ctx* c, int32_t i, int64_t* out) {
    if (!c || !out || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    const InstHost& in = c->inst[i];
    if (in.rec_t.empty()) return GSBS_OK;
    std::vector<long long> buf((size_t)c->max_rec * kMaxSpecies);
    HIPCHK(hipMemcpyAsync(buf.data(), c->rec + (size_t)i * c->max_rec * kMaxSpecies, sizeof(long long) * buf.size(),
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (size_t r = 0; r < in.rec_t.size(); ++r)
        for (int s = 0; s < c->ns; ++s) out[r * c->ns + s] = buf[r * kMaxSpecies + s];
    return GSBS_OK;
}

int gsbs_get_gvalues(gsbs_ctx* c, int32_t i, double* out) {
    if (!c || !out || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    const InstHost& in = c->inst[i];
    std::vector<int64_t> cnt(in.rec_t.size() * (size_t)c->ns);
    CHK(gsbs_get_counts(c, i, cnt.data()));
    for (size_t r = 0; r < in.rec_t.size(); ++r)
        for (int s = 0; s < c->ns; ++s) {
            const double e = in.rec_edep[r];
            const int64_t v = cnt[r * c->ns + s];
            out[r * c->ns + s] = (in.rec_done[r] && e > 0 && v >= 0) ? (double)v / (e / 100.0) : NAN;
        }
    return GSBS_OK;
}

int gsbs_get_current_counts(gsbs_ctx* c, int32_t i, int64_t* out) {
    if (!c || !out || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    std::vector<long long> buf(kMaxSpecies);
    HIPCHK(hipMemcpyAsync(buf.data(), c->counts + (size_t)i * kMaxSpecies, sizeof(long long) * kMaxSpecies,
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int s = 0; s < c->ns; ++s) out[s] = buf[s];
    return GSBS_OK;
}

// ------------------------------------------------------------ surrogate ---
namespace {

// Reference subsample, pair-correlation shell counts and shell volumes of
// instance i (device), for the current state.
int sur_pair_counts(gsbs_ctx* c, int i, double r_max, int n_ref_max, std::vector<long long>& cnt) {
    InstHost& in = c->inst[i];
    const int nr = (int)c->rx.size();
    cnt.assign(kMaxSpecies, 0);
    HIPCHK(hipMemcpyAsync(cnt.data(), c->counts + (size_t)i * kMaxSpecies, sizeof(long long) * kMaxSpecies,
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const int cap = 2 * n_ref_max + 64;
    if (cap > c->sur_cap) {
        dfree(c->sur_ref_idx);
        CHK(dalloc(&c->sur_ref_idx, (size_t)kMaxSpecies * cap));
        c->sur_cap = cap;
    }
    if (!c->sur_ref_cnt) {
        CHK(dalloc(&c->sur_ref_cnt, kMaxSpecies));
        CHK(dalloc(&c->sur_pair_ab, 2 * kMaxReactions));
        CHK(dalloc(&c->sur_edges2, (size_t)kMaxReactions * (kSurBins + 1)));
        CHK(dalloc(&c->sur_shell, (size_t)kMaxReactions * kSurBins));
        CHK(dalloc(&c->sur_hist, (size_t)kMaxReactions * kSurBins));
        CHK(dalloc(&c->sur_vec, 3 * (size_t)kFeatures));
        CHK(dalloc(&c->sur_newc, kMaxSpecies));
    }
    SurStrides st{};
    for (int s = 0; s < kMaxSpecies; ++s)
        st.s[s] = (int32_t)std::max<long long>(1, (cnt[s] + n_ref_max - 1) / std::max(n_ref_max, 1));
    // log-spaced shells from R to r_max: e_k = R (r_max / R)^(k / 32)
    std::vector<int32_t> ab(2 * nr);
    std::vector<float> e2((size_t)nr * (kSurBins + 1));
    std::vector<double> vol((size_t)nr * kSurBins);
    const double rmax = std::min(0.5 * in.L, r_max);
    for (int r = 0; r < nr; ++r) {
        ab[2 * r] = c->rx[r].a;
        ab[2 * r + 1] = c->rx[r].b;
        const double R = std::min(c->R[r], 0.5 * rmax);
        std::vector<double> e(kSurBins + 1);
        for (int k = 0; k <= kSurBins; ++k) e[k] = R * std::pow(rmax / R, (double)k / kSurBins);
        for (int k = 0; k <= kSurBins; ++k) e2[(size_t)r * (kSurBins + 1) + k] = (float)(e[k] * e[k]);
        const double f = 4.0 / 3.0 * 3.14159265358979323846;
        for (int k = 0; k < kSurBins; ++k)
            vol[(size_t)r * kSurBins + k] = f * (k == 0 ? e[1] * e[1] * e[1] : e[k + 1] * e[k + 1] * e[k + 1] - e[k] * e[k] * e[k]);
    }
    HIPCHK(hipMemcpyAsync(c->sur_pair_ab, ab.data(), sizeof(int32_t) * ab.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->sur_edges2, e2.data(), sizeof(float) * e2.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->sur_shell, vol.data(), sizeof(double) * vol.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemsetAsync(c->sur_ref_cnt, 0, sizeof(int32_t) * kMaxSpecies, c->st));
    HIPCHK(hipMemsetAsync(c->sur_hist, 0, sizeof(unsigned long long) * nr * kSurBins, c->st));
    int64_t n_all = 0;
    for (auto& q : c->inst) n_all += q.n_est;
    launch_collect_refs(c->st, c->pos[c->cur], c->uid[c->cur], c->ctr, i, st, cap, c->sur_ref_idx, c->sur_ref_cnt,
                        &c->ctr->err, grid_for(std::max<int64_t>(n_all, 1)));
    launch_pair_corr(c->st, c->pos[c->cur], c->ctr, i, c->sur_ref_idx, c->sur_ref_cnt, cap, c->sur_pair_ab,
                     c->sur_edges2, nr, (float)in.L, c->sur_hist, n_all);
    HIPCHK(hipGetLastError());
    return GSBS_OK;
}

}  // namespace

int gsbs_features(gsbs_ctx* c, int32_t i, double dt_next_ns, double r_max_nm, int32_t n_ref_max, double c_floor_M,
                  const float* mu, const float* sd, float* out, int32_t out_is_device) {
    if (!c || !out || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    if (!c->chem_ready || c->ns != 7 || c->rx.size() != 9)
        return fail(GSBS_ESTATE, "features are defined for 7 species and 9 reactions");
    if (!(dt_next_ns > 0) || !(r_max_nm > 0) || n_ref_max < 1 || !(c_floor_M > 0))
        return fail(GSBS_EINVAL, "bad feature parameters");
    std::vector<long long> cnt;
    CHK(sur_pair_counts(c, i, r_max_nm, n_ref_max, cnt));
    int32_t rc[kMaxSpecies];
    HIPCHK(hipMemcpyAsync(rc, c->sur_ref_cnt, sizeof(rc), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int s = 0; s < kMaxSpecies; ++s)
        if (rc[s] > c->sur_cap) return fail(GSBS_ECAPACITY, "reference subsample above its capacity");
    std::vector<float> ms(2 * kFeatures);
    for (int f = 0; f < kFeatures; ++f) {
        ms[f] = mu ? mu[f] : 0.0f;
        ms[kFeatures + f] = sd ? sd[f] : 1.0f;
    }
    HIPCHK(hipMemcpyAsync(c->sur_vec, ms.data(), sizeof(float) * ms.size(), hipMemcpyHostToDevice, c->st));
    float* dst = out_is_device ? out : c->sur_vec + 2 * kFeatures;
    launch_features(c->st, c->counts, i, c->ns, c->sur_hist, c->sur_ref_cnt, c->sur_cap, c->sur_pair_ab, c->sur_shell,
                    (int)c->rx.size(), c->inst[i].L, dt_next_ns, c_floor_M, c->sur_vec, c->sur_vec + kFeatures,
                    (mu || sd) ? 1 : 0, dst);
    HIPCHK(hipGetLastError());
    if (!out_is_device) {
        HIPCHK(hipMemcpyAsync(out, dst, sizeof(float) * kFeatures, hipMemcpyDeviceToHost, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    return check_device_errors(c);
}

int gsbs_pair_corr(gsbs_ctx* c, int32_t i, double r_max_nm, int32_t n_ref_max, float* out) {
    if (!c || !out) return fail(GSBS_EINVAL, "null");
    std::vector<float> row(kFeatures);
    CHK(gsbs_features(c, i, 1.0, r_max_nm, n_ref_max, 1e-10, nullptr, nullptr, row.data(), 0));
    std::copy(row.begin() + 7, row.begin() + 7 + 9 * kSurBins, out);
    return GSBS_OK;
}

// Reaction table of the rate equations (see gsbs_numodes).
static void build_ode_table(const gsbs_ctx* c, OdeTable& tb) {
    tb.ns = c->ns;
    tb.nr = (int32_t)c->rx.size();
    for (int r = 0; r < tb.nr; ++r) {
        const gsbs_reaction& q = c->rx[r];
        tb.ra[r] = q.a;
        tb.rb[r] = q.b;
        // 1e10 L/mol/s -> L/mol/ns; the printed k of a self-recombination is 2k
        tb.kr[r] = 10.0 * q.k_in * (q.a == q.b ? 0.5 : 1.0);
        tb.nu[r][q.a] -= 1.0;
        if (!q.keep_b) tb.nu[r][q.b] -= 1.0;
        for (int k = 0; k < q.n_products; ++k) tb.nu[r][q.products[k]] += 1.0;
    }
    for (const gsbs_first_order& f : c->fo) {
        const int r = tb.nr++;
        tb.ra[r] = f.a;
        tb.rb[r] = -1;
        tb.kr[r] = f.k_per_ns;
        tb.nu[r][f.a] -= 1.0;
        for (int k = 0; k < f.n_products; ++k) tb.nu[r][f.products[k]] += 1.0;
    }
    for (const gsbs_source& q : c->src)
        for (int k = 0; k < q.n_products; ++k) tb.src[q.products[k]] += q.rate_M_per_ns;
}

// Checks shared by the two rate-equation entry points.
static int numodes_args(gsbs_ctx* c, int32_t n, int32_t n_species, const double* c0, const double* dt_ns,
                        double* c1, double rtol) {
    if (!c || n < 0 || (n > 0 && (!c0 || !dt_ns || !c1)) || !(rtol > 0.0) || rtol > 0.1)
        return fail(GSBS_EINVAL, "bad rate-equation arguments");
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    if (n_species != c->ns) return fail(GSBS_EINVAL, "rate equations: n_species is not the table's");
    if (c->ns > kOdeMaxSpecies) return fail(GSBS_EINVAL, "the rate equations take at most 8 species");
    if (c->rx.size() + c->fo.size() > (size_t)kMaxReactions)
        return fail(GSBS_EINVAL, "the rate equations take at most 32 reactions and channels");
    return GSBS_OK;
}

int gsbs_numodes_noalloc(gsbs_ctx* c, int32_t n, int32_t n_species, const double* c0, const double* dt_ns,
                         double* c1, double rtol, int32_t* steps) {
    CHK(numodes_args(c, n, n_species, c0, dt_ns, c1, rtol));
    if (n > 0 && !steps) return fail(GSBS_EINVAL, "steps: a host array of n entries is required");
    if (n > kNoAllocMaxMixtures) return fail(GSBS_EINVAL, "gsbs_numodes_noalloc: at most 1048576 mixtures per call");
    if (n == 0) return GSBS_OK;
    OdeTable tb{};
    build_ode_table(c, tb);
    int32_t* sc = nullptr;
    CHK(numodes_scratch(&sc));
    launch_numodes(c->st, c0, dt_ns, c1, sc, n, tb, rtol, 1e-10 * rtol, 200000);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(steps, sc, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int32_t m = 0; m < n; ++m)
        if (steps[m] < 0) return fail(GSBS_ESTATE, "rate equations: step limit reached");
    return GSBS_OK;
}

int gsbs_numodes(gsbs_ctx* c, int32_t n, int32_t n_species, const double* c0, const double* dt_ns, double* c1,
                 double rtol, int32_t* steps, int32_t on_device) {
    CHK(numodes_args(c, n, n_species, c0, dt_ns, c1, rtol));
    if (n == 0) return GSBS_OK;
    OdeTable tb{};
    build_ode_table(c, tb);
    const size_t nc = (size_t)n * (size_t)c->ns;
    double *d0 = nullptr, *dd = nullptr, *d1 = nullptr;
    int32_t* dsteps = nullptr;
    struct Release {
        double **a, **b, **d;
        int32_t** s;
        ~Release() {
            dfree(*a);
            dfree(*b);
            dfree(*d);
            dfree(*s);
        }
    } release{&d0, &dd, &d1, &dsteps};
    const double* pc0 = c0;
    const double* pdt = dt_ns;
    double* pc1 = c1;
    CHK(dalloc(&dsteps, (size_t)n));
    if (!on_device) {
        CHK(dalloc(&d0, nc));
        CHK(dalloc(&dd, (size_t)n));
        CHK(dalloc(&d1, nc));
        HIPCHK(hipMemcpyAsync(d0, c0, sizeof(double) * nc, hipMemcpyHostToDevice, c->st));
        HIPCHK(hipMemcpyAsync(dd, dt_ns, sizeof(double) * n, hipMemcpyHostToDevice, c->st));
        pc0 = d0;
        pdt = dd;
        pc1 = d1;
    }
    launch_numodes(c->st, pc0, pdt, pc1, dsteps, n, tb, rtol, 1e-10 * rtol, 200000);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> hs((size_t)n);
    HIPCHK(hipMemcpyAsync(hs.data(), dsteps, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->st));
    if (!on_device) HIPCHK(hipMemcpyAsync(c1, d1, sizeof(double) * nc, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (steps) std::copy(hs.begin(), hs.end(), steps);
    for (int32_t m = 0; m < n; ++m)
        if (hs[(size_t)m] < 0) return fail(GSBS_ESTATE, "rate equations: step limit reached");
    return GSBS_OK;
}

int gsbs_ssa(gsbs_ctx* c, int32_t n, int32_t n_species, const int32_t* n0, const double* volume_L, int32_t n_rec,
             const double* t_rec_ns, uint64_t seed, uint64_t stream0, int64_t max_events, int32_t* out,
             int64_t* events, int32_t on_device) {
    if (!c || n < 0 || n_rec < 1 || !t_rec_ns || max_events < 0 || (n > 0 && (!n0 || !volume_L || !out)))
        return fail(GSBS_EINVAL, "bad stochastic-kinetics arguments");
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    if (n_species != c->ns) return fail(GSBS_EINVAL, "stochastic kinetics: n_species is not the table's");
    if (c->ns > kOdeMaxSpecies || (int)c->rx.size() > kSsaMaxReactions)
        return fail(GSBS_EINVAL, "stochastic kinetics take at most 8 species and 16 reactions");
    for (int32_t k = 0; k < n_rec; ++k)
        if (!(t_rec_ns[k] >= 0.0) || !std::isfinite(t_rec_ns[k]) || (k > 0 && t_rec_ns[k] < t_rec_ns[k - 1]))
            return fail(GSBS_EINVAL, "record times must be finite, >= 0 and ascending");
    if (!on_device)
        for (int32_t m = 0; m < n; ++m) {
            if (!(volume_L[m] > 0.0) || !std::isfinite(volume_L[m])) return fail(GSBS_EINVAL, "bad volume");
            for (int s = 0; s < c->ns; ++s)
                if (n0[(size_t)m * c->ns + s] < 0) return fail(GSBS_EINVAL, "negative initial count");
        }
    if (n == 0) return GSBS_OK;
    SsaTable tb{};
    tb.ns = c->ns;
    tb.nr = (int32_t)c->rx.size();
    for (int r = 0; r < tb.nr; ++r) {
        const gsbs_reaction& q = c->rx[r];
        int nu[kOdeMaxSpecies] = {};
        nu[q.a] -= 1;
        if (!q.keep_b) nu[q.b] -= 1;
        for (int k = 0; k < q.n_products; ++k) nu[q.products[k]] += 1;
        tb.ra[r] = q.a;
        tb.rb[r] = q.b;
        tb.k10[r] = 10.0 * q.k_in;  // 1e10 L/mol/s -> L/mol/ns
        uint64_t d = 0;
        for (int s = 0; s < kOdeMaxSpecies; ++s) d |= (uint64_t)(uint8_t)(int8_t)nu[s] << (8 * s);
        tb.dn[r] = d;
    }
    tb.nfo = (int32_t)c->fo.size();
    for (int q = 0; q < tb.nfo; ++q) {
        // the oracle's order: channels by species
        int nu[kOdeMaxSpecies] = {};
        const gsbs_first_order& f = c->fo[(size_t)q];
        nu[f.a] -= 1;
        for (int k = 0; k < f.n_products; ++k) nu[f.products[k]] += 1;
        uint64_t d = 0;
        for (int s = 0; s < kOdeMaxSpecies; ++s) d |= (uint64_t)(uint8_t)(int8_t)nu[s] << (8 * s);
        tb.fo_a[q] = f.a;
        tb.fo_k[q] = f.k_per_ns;
        tb.dn[kSsaMaxReactions + q] = d;
    }
    tb.nsrc = (int32_t)c->src.size();
    for (int q = 0; q < tb.nsrc; ++q) {
        int nu[kOdeMaxSpecies] = {};
        for (int k = 0; k < c->src[q].n_products; ++k) nu[c->src[q].products[k]] += 1;
        uint64_t d = 0;
        for (int s = 0; s < kOdeMaxSpecies; ++s) d |= (uint64_t)(uint8_t)(int8_t)nu[s] << (8 * s);
        tb.src_rate[q] = c->src[q].rate_M_per_ns;
        tb.dn[kSsaMaxReactions + kOdeMaxSpecies + q] = d;
    }
    const size_t nc = (size_t)n * (size_t)c->ns, no = (size_t)n * (size_t)n_rec * (size_t)c->ns;
    int32_t *d0 = nullptr, *dout = nullptr;
    double *dvol = nullptr, *drec = nullptr;
    long long* dev = nullptr;
    struct Release {
        int32_t **a, **b;
        double **v, **r;
        long long** e;
        ~Release() {
            dfree(*a);
            dfree(*b);
            dfree(*v);
            dfree(*r);
            dfree(*e);
        }
    } release{&d0, &dout, &dvol, &drec, &dev};
    const int32_t* p0 = n0;
    const double* pv = volume_L;
    int32_t* po = out;
    CHK(dalloc(&drec, (size_t)n_rec));
    CHK(dalloc(&dev, (size_t)n));
    HIPCHK(hipMemcpyAsync(drec, t_rec_ns, sizeof(double) * n_rec, hipMemcpyHostToDevice, c->st));
    if (!on_device) {
        CHK(dalloc(&d0, nc));
        CHK(dalloc(&dvol, (size_t)n));
        CHK(dalloc(&dout, no));
        HIPCHK(hipMemcpyAsync(d0, n0, sizeof(int32_t) * nc, hipMemcpyHostToDevice, c->st));
        HIPCHK(hipMemcpyAsync(dvol, volume_L, sizeof(double) * n, hipMemcpyHostToDevice, c->st));
        p0 = d0;
        pv = dvol;
        po = dout;
    }
    launch_ssa(c->st, p0, pv, drec, n_rec, po, dev, n, tb, seed, stream0, (long long)max_events);
    HIPCHK(hipGetLastError());
    std::vector<long long> he((size_t)n);
    HIPCHK(hipMemcpyAsync(he.data(), dev, sizeof(long long) * n, hipMemcpyDeviceToHost, c->st));
    if (!on_device) HIPCHK(hipMemcpyAsync(out, dout, sizeof(int32_t) * no, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (events)
        for (int32_t m = 0; m < n; ++m) events[m] = (int64_t)he[(size_t)m];
    for (int32_t m = 0; m < n; ++m)
        if (he[(size_t)m] < 0) return fail(GSBS_ESTATE, "stochastic kinetics: event limit reached");
    return GSBS_OK;
}

int gsbs_repopulate(gsbs_ctx* c, int32_t i, double t_new, const float* y, int32_t y_is_device, const float* mu_y,
                    const float* sd_y, double c_floor_M, int32_t relative) {
    if (!c || !y || !mu_y || !sd_y || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad arguments");
    if (c->broken) return fail(GSBS_ESTATE, kBroken);
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    InstHost& in = c->inst[i];
    if (!(t_new >= in.t)) return fail(GSBS_ESTATE, "re-population before the instance's present time");
    for (auto& p : in.pending)
        if (p.t < t_new) return fail(GSBS_ESTATE, "an injection falls before the re-population time");
    if (!(c_floor_M > 0)) return fail(GSBS_EINVAL, "bad concentration floor");
    if (!c->sur_vec) {
        std::vector<long long> tmp;
        CHK(sur_pair_counts(c, i, 1.0, 1, tmp));  // allocates the buffers
    }
    // staging: mu_y, sd_y and y in the 3 rows of sur_vec
    std::vector<float> ms(2 * kFeatures, 0.0f);
    for (int s = 0; s < c->ns; ++s) {
        ms[s] = mu_y[s];
        ms[kFeatures + s] = sd_y[s];
    }
    HIPCHK(hipMemcpyAsync(c->sur_vec, ms.data(), sizeof(float) * ms.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->sur_vec + 2 * kFeatures, y, sizeof(float) * c->ns,
                          y_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
    const double vol_litre = in.L * in.L * in.L * 1e-24;
    launch_repop_counts(c->st, c->sur_vec + 2 * kFeatures, c->sur_vec, c->sur_vec + kFeatures, c->ns, c_floor_M,
                        vol_litre, c->seed, i, in.step, relative ? 1 : 0, c->counts, c->sur_newc);
    std::vector<long long> nc(kMaxSpecies, 0);
    HIPCHK(hipMemcpyAsync(nc.data(), c->sur_newc, sizeof(long long) * kMaxSpecies, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    int64_t total = 0;
    for (int s = 0; s < c->ns; ++s) total += nc[s];
    if (total > 0x3FFFFFFF) return fail(GSBS_ECAPACITY, "re-population count too large");
    DevCounters h{};
    CHK(read_counters(c, &h));
    CHK(ensure_capacity(c, (int64_t)h.n_in + total + 1024));
    int64_t n_all = 0;
    for (auto& q : c->inst) n_all += q.n_est;
    launch_repop(c->st, c->pos[c->cur], c->uid[c->cur], c->ctr, c->sur_newc, c->ns, (int)total, i, in.next_uid,
                 c->seed, in.step, (float)in.L, c->cap, c->counts, grid_for(std::max<int64_t>(n_all + total, 1)));
    HIPCHK(hipGetLastError());
    in.next_uid += (uint64_t)total;
    // records strictly between the old and the new time are not taken
    for (size_t r = 0; r < in.rec_t.size(); ++r)
        if (!in.rec_done[r] && in.rec_t[r] > in.t && in.rec_t[r] < t_new) in.rec_done[r] = 1;
    in.t = t_new;
    in.n_est = total;
    for (int s = 0; s < kMaxSpecies; ++s) in.sp_est[s] = nc[s];
    HIPCHK(hipStreamSynchronize(c->st));
    return check_device_errors(c);
}

int gsbs_get_time(gsbs_ctx* c, int32_t i, double* t) {
    if (!c || !t || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    *t = c->inst[i].t;
    return GSBS_OK;
}

int gsbs_get_n(gsbs_ctx* c, int32_t i, int64_t* n) {
    if (!c || !n || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad instance");
    std::vector<int64_t> cnt(c->ns);
    CHK(gsbs_get_current_counts(c, i, cnt.data()));
    int64_t s = 0;
    for (auto v : cnt) s += v;
    *n = s;
    return GSBS_OK;
}

int gsbs_get_stats(gsbs_ctx* c, gsbs_stats* out) {
    if (!c || !out) return fail(GSBS_EINVAL, "null");
    DevCounters h{};
    CHK(read_counters(c, &h));
    std::vector<unsigned long long> ms(c->n_inst);
    HIPCHK(hipMemcpyAsync(ms.data(), c->msteps, sizeof(unsigned long long) * c->n_inst, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    out->steps = c->steps;
    out->molecule_steps = 0;
    for (auto v : ms) out->molecule_steps += (int64_t)v;
    out->reactions = (int64_t)h.reactions;
    out->pair_candidates = (int64_t)h.cand;
    out->max_live = c->max_live;
    return GSBS_OK;
}

int gsbs_get_device_bytes(gsbs_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return fail(GSBS_EINVAL, "null");
    int64_t b = 0;
    const int64_t cap = c->cap;
    b += 2 * cap * (int64_t)(sizeof(float4) + sizeof(uint64_t));                       // pos, uid (ping-pong)
    b += cap * (int64_t)(sizeof(float4) + sizeof(uint2) + sizeof(unsigned long long) + sizeof(int32_t) +
                         2 * sizeof(float4));                                           // pos0, cellrank, claim, mate, x0, xnew
    b += (int64_t)(c->cell_cap + 1) * 2 * (int64_t)sizeof(uint32_t) +
         (int64_t)(c->cell_cap / 4096 + 2) * (int64_t)sizeof(unsigned long long);       // cells, scan status
    b += (int64_t)c->pair_cap * (int64_t)sizeof(PairRec);
    b += (int64_t)c->n_inst * c->max_rec * kMaxSpecies * (int64_t)sizeof(long long);
    for (const auto& in : c->inst)
        for (const auto& p : in.pending) b += p.n * (int64_t)(3 * sizeof(float) + 1);
    *bytes = b;
    return GSBS_OK;
}

int gsbs_set_profiling(gsbs_ctx* c, int32_t on) {
    if (!c) return fail(GSBS_EINVAL, "null");
    if (on && !c->prof_ev[0])
        for (auto& e : c->prof_ev) HIPCHK(hipEventCreate(&e));
    c->profiling = on != 0;
    c->step_log.clear();
    for (int k = 0; k < kStepKernels; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
        c->prof_work[k] = 0;
        c->prof_cnd[k] = 0;
    }
    if (on) {
        DevCounters h{};
        HIPCHK(hipMemcpy(&h, c->ctr, sizeof(h), hipMemcpyDeviceToHost));
        c->prof_cand = h.cand;
    }
    return GSBS_OK;
}

int gsbs_get_tuning(int32_t max_k, int32_t* keys, int32_t* best, double* best_ms, int32_t* n) {
    if (!n) return fail(GSBS_EINVAL, "null");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int32_t k = 0;
    for (const auto& kv : g_tune) {
        int b = -1;
        double bt = 0.0;
        for (int q = 0; q < kNumCfg; ++q) {
            if (kv.second.cnt[q] == 0) continue;
            const double t = kv.second.ms[q] / kv.second.cnt[q];
            if (b < 0 || t < bt) {
                b = q;
                bt = t;
            }
        }
        if (b < 0) continue;
        if (k < max_k) {
            if (keys) {
                keys[2 * k] = kv.first.first;
                keys[2 * k + 1] = kv.first.second;
            }
            if (best) best[k] = b;
            if (best_ms) best_ms[k] = bt;
        }
        ++k;
    }
    *n = k;
    return GSBS_OK;
}

int gsbs_get_step_log(gsbs_ctx* c, int64_t max_n, int64_t* step, double* ms, int32_t* grid, int64_t* n_est,
                      int64_t* n) {
    if (!c || !n) return fail(GSBS_EINVAL, "null");
    const int64_t m = (int64_t)c->step_log.size();
    for (int64_t k = 0; k < std::min(m, max_n); ++k) {
        const auto& e = c->step_log[(size_t)k];
        if (step) step[k] = e.step;
        if (ms) ms[k] = e.ms;
        if (grid) {
            grid[4 * k] = e.nc;
            grid[4 * k + 1] = e.reach;
            grid[4 * k + 2] = e.by_species;
            grid[4 * k + 3] = e.cfg;
        }
        if (n_est) n_est[k] = e.n_est;
    }
    *n = m;
    return GSBS_OK;
}

int gsbs_set_live_timing(gsbs_ctx* c, uint32_t kernel_mask) {
    if (!c || (kernel_mask >> kStepKernels) != 0u) return fail(GSBS_EINVAL, "kernel mask: bits 0..5");
    HIPCHK(hipStreamSynchronize(c->st));
    for (int b = 0; b < 2; ++b) CHK(live_harvest(c, b));
    if (kernel_mask && c->live_ev[0].empty()) {
        for (int b = 0; b < 2; ++b) {
            c->live_ev[b].assign((size_t)kChunk * (kStepKernels + 1), nullptr);
            for (auto& e : c->live_ev[b]) HIPCHK(hipEventCreate(&e));
            HIPCHK(hipEventCreateWithFlags(&c->live_done[b], hipEventDisableTiming));
        }
    }
    c->live_mask = kernel_mask;
    c->live_bins = 0;
    for (int k = 0; k < kStepKernels; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
        c->prof_work[k] = 0;
        c->prof_cnd[k] = 0;
    }
    return read_counters(c, &c->live_base);
}

int gsbs_get_profile(gsbs_ctx* c, int32_t max_k, char* names, double* total_ms, int64_t* launches, int64_t* work,
                     int64_t* candidates, int32_t* n) {
    if (!c || !n) return fail(GSBS_EINVAL, "null");
    if (c->live_mask && !c->profiling) {
        // work units of the live-timed steps from the device's cumulative counters
        DevCounters h{};
        CHK(read_counters(c, &h));
        const int64_t all = (int64_t)(h.msteps_mode[0] + h.msteps_mode[1]) -
                            (int64_t)(c->live_base.msteps_mode[0] + c->live_base.msteps_mode[1]);
        const int64_t whole = (int64_t)(h.msteps_mode[0] - c->live_base.msteps_mode[0]);
        const int64_t sp = (int64_t)(h.msteps_mode[1] - c->live_base.msteps_mode[1]);
        const int64_t csp = (int64_t)(h.cand_sp - c->live_base.cand_sp);
        const int64_t call = (int64_t)(h.cand - c->live_base.cand);
        for (int k = 0; k < kStepKernels; ++k) {
            c->prof_work[k] = k == 1 ? c->live_bins : (k == 3 ? whole : (k == 4 ? sp : all));
            c->prof_cnd[k] = k == 3 ? call - csp : (k == 4 ? csp : 0);
        }
    }
    for (int k = 0; k < std::min(max_k, kStepKernels); ++k) {
        if (names) {
            std::memset(names + 32 * k, 0, 32);
            std::strncpy(names + 32 * k, kStepKernelNames[k], 31);
        }
        if (total_ms) total_ms[k] = c->prof_ms[k];
        if (launches) launches[k] = c->prof_n[k];
        if (work) work[k] = c->prof_work[k];
        if (candidates) candidates[k] = c->prof_cnd[k];
    }
    *n = kStepKernels;
    return GSBS_OK;
}

int gsbs_plan_schedule(double t_start, double t_end, int32_t n_anchor, const double* anchors, int32_t n_events,
                       const double* events, double dt0, double ratio, double dt_max, double* out, int64_t max_out,
                       int64_t* n_out) {
    if (!n_out || n_anchor < 0 || n_events < 0 || (n_anchor && !anchors) || (n_events && !events) ||
        !(dt0 > 0) || !(ratio > 1) || !(dt_max > 0) || t_end < t_start)
        return fail(GSBS_EINVAL, "bad schedule arguments");
    std::vector<double> s;
    plan_steps(t_start, t_end, anchors, n_anchor, events, n_events, dt0, ratio, dt_max, s);
    *n_out = (int64_t)s.size();
    if (out)
        for (int64_t k = 0; k < std::min<int64_t>(max_out, (int64_t)s.size()); ++k) out[k] = s[k];
    return GSBS_OK;
}

// ---------------------------------------------------------------- debug ---

int gsbs_debug_get_state(gsbs_ctx* c, int32_t i, int64_t max_n, float* xyz, uint8_t* sp, uint64_t* uid,
                         int64_t* n) {
    if (!c || !n || i < 0 || i >= c->n_inst) return fail(GSBS_EINVAL, "bad arguments");
    DevCounters h{};
    CHK(read_counters(c, &h));
    std::vector<float4> p(h.n_in);
    std::vector<uint64_t> u(h.n_in);
    if (h.n_in > 0) {
        HIPCHK(hipMemcpyAsync(p.data(), c->pos[c->cur], sizeof(float4) * h.n_in, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(u.data(), c->uid[c->cur], sizeof(uint64_t) * h.n_in, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    int64_t k = 0;
    for (int32_t q = 0; q < h.n_in; ++q) {
        int meta;
        std::memcpy(&meta, &p[q].w, 4);
        if ((meta & 0xFF) == kDead || (meta >> 8) != i) continue;
        if (k < max_n) {
            if (xyz) {
                xyz[3 * k] = p[q].x;
                xyz[3 * k + 1] = p[q].y;
                xyz[3 * k + 2] = p[q].z;
            }
            if (sp) sp[k] = (uint8_t)(meta & 0xFF);
            if (uid) uid[k] = u[q];
        }
        ++k;
    }
    *n = k;
    return GSBS_OK;
}

int gsbs_debug_set_state(gsbs_ctx* c, int64_t n, const float* xyz, const uint8_t* sp, const uint64_t* uid,
                         int64_t step, uint64_t next_uid) {
    if (!c || n < 0 || (n > 0 && (!xyz || !sp || !uid))) return fail(GSBS_EINVAL, "bad state");
    if (c->n_inst != 1) return fail(GSBS_EINVAL, "debug state needs a single-instance context");
    if (c->ns == 0) return fail(GSBS_ESTATE, "set the species first");
    CHK(ensure_capacity(c, n + n / 2 + 1024));
    std::vector<float4> p(n);
    std::vector<long long> cnt(kMaxSpecies, 0);
    for (int64_t k = 0; k < n; ++k) {
        if (sp[k] >= c->ns) return fail(GSBS_EINVAL, "species index out of range");
        int meta = sp[k];
        float w;
        std::memcpy(&w, &meta, 4);
        p[k] = make_float4(xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2], w);
        cnt[sp[k]]++;
    }
    c->cur = 0;
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(c->pos[0], p.data(), sizeof(float4) * n, hipMemcpyHostToDevice, c->st));
        HIPCHK(hipMemcpyAsync(c->uid[0], uid, sizeof(uint64_t) * n, hipMemcpyHostToDevice, c->st));
    }
    HIPCHK(hipMemcpyAsync(c->counts, cnt.data(), sizeof(long long) * kMaxSpecies, hipMemcpyHostToDevice, c->st));
    DevCounters h{};
    CHK(read_counters(c, &h));
    h.n_in = (int32_t)n;
    h.n_live = (int32_t)n;
    h.n_pairs = 0;
    h.err = 0;
    HIPCHK(hipMemcpyAsync(c->ctr, &h, sizeof(DevCounters), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    InstHost& in = c->inst[0];
    in.step = (uint64_t)step;
    in.next_uid = next_uid;
    in.n_est = n;
    for (int k = 0; k < kMaxSpecies; ++k) in.sp_est[k] = cnt[k];
    return GSBS_OK;
}

int gsbs_debug_step(gsbs_ctx* c, double dt, int32_t flags, const float* xyz0, int32_t nc_force) {
    if (!c || !(dt > 0)) return fail(GSBS_EINVAL, "bad step");
    if (c->n_inst != 1) return fail(GSBS_EINVAL, "debug step needs a single-instance context");
    if (!c->chem_ready) return fail(GSBS_ESTATE, "set species and reactions first");
    DevCounters h{};
    CHK(read_counters(c, &h));
    if ((flags & kStepFixed)) {
        if (!xyz0) return fail(GSBS_EINVAL, "fixed-position step needs start positions");
        std::vector<float4> p(h.n_in);
        for (int32_t k = 0; k < h.n_in; ++k) p[k] = make_float4(xyz0[3 * k], xyz0[3 * k + 1], xyz0[3 * k + 2], 0.f);
        if (h.n_in)
            HIPCHK(hipMemcpyAsync(c->x0_dbg, p.data(), sizeof(float4) * h.n_in, hipMemcpyHostToDevice, c->st));
    }
    if (flags & kStepLogAll) CHK(ensure_pairs(c, 1u << 24));
    InstHost& in = c->inst[0];
    in.n_est = std::max<int64_t>(h.n_in, 1);
    InstStep* S = c->h_chunk[c->chunk_buf];
    HIPCHK(hipEventSynchronize(c->chunk_ev[c->chunk_buf]));
    if (nc_force > 0) {
        double rcmax = 0.0;
        for (size_t r = 0; r < c->rx.size(); ++r) {
            const double Dab = c->D[c->rx[r].a] + c->D[c->rx[r].b];
            rcmax = std::max(rcmax, cutoff_of(c->R[r], Dab, dt, c->prm.c_cut));
        }
        (void)rcmax;
        if (nc_force > 1024) return fail(GSBS_EINVAL, "forced search grid too fine");
    }
    const double rcmax = fill_physics(c, in.L, in.step, 0, dt, true, S[0]);
    int cfg = default_cfg(tune_key(in.L, in.n_est, rcmax).first);
    if (c->prm.grid_config >= 0) cfg = c->prm.grid_config;
    GridCfg gc = kCfgs[cfg];
    if (flags & kStepBySpecies) gc.by_species = 1;
    if (flags & kStepWholeCells) gc.by_species = 0;
    S[0].bin_base = 0;
    const int32_t ncell = fill_grid(c, in.sp_est, in.L, in.n_est, rcmax, gc, nc_force, S[0]);
    assign_splits(c, S, 1);
    S[0].unit_base = 0;
    const int32_t units = (int32_t)units_of(S[0], c->ns);
    const int32_t cells = S[0].by_species ? ncell * c->ns : ncell;
    CHK(ensure_cells(c, (int64_t)cells));
    HIPCHK(hipMemcpyAsync(c->d_chunk[c->chunk_buf], S, sizeof(InstStep), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipEventRecord(c->chunk_ev[c->chunk_buf], c->st));
    StepBuffers bf = buffers(c);
    flags |= S[0].by_species ? kStepHasSpecies : kStepHasWhole;
    CHK(run_step(c, bf, c->d_chunk[c->chunk_buf], 1, cells, units, grid_for(h.n_in), flags));
    c->chunk_buf ^= 1;
    c->cur ^= 1;
    c->dbg_nc = S[0].nc;
    c->dbg_cell_base = 0;
    c->dbg_by_species = S[0].by_species;
    if (!(flags & kStepSearchOnly)) {
        in.step++;
        in.t += dt;
        c->steps++;
    }
    HIPCHK(hipStreamSynchronize(c->st));
    CHK(check_device_errors(c));
    return refresh_estimates(c);
}

int gsbs_debug_get_pairs(gsbs_ctx* c, int64_t max_n, uint64_t* uid2, float* P, uint32_t* u24, int32_t* rx,
                         int32_t* flags, int64_t* n) {
    if (!c || !n) return fail(GSBS_EINVAL, "null");
    DevCounters h{};
    CHK(read_counters(c, &h));
    const int64_t np = std::min<int64_t>(h.n_pairs, c->pair_cap);
    std::vector<PairRec> pr(np);
    std::vector<uint64_t> u(std::max<int32_t>(h.n_live, 1));
    if (np > 0) {
        HIPCHK(hipMemcpyAsync(pr.data(), c->pairs, sizeof(PairRec) * np, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(u.data(), c->uid[c->cur], sizeof(uint64_t) * h.n_live, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    for (int64_t k = 0; k < std::min(np, max_n); ++k) {
        const uint64_t a = u[pr[k].i], b = u[pr[k].j];
        if (uid2) {
            uid2[2 * k] = a < b ? a : b;
            uid2[2 * k + 1] = a < b ? b : a;
        }
        if (P) P[k] = pr[k].P;
        if (u24) u24[k] = pr[k].u24;
        if (rx) rx[k] = pr[k].rx;
        if (flags) flags[k] = pr[k].flags;
    }
    *n = np;
    return GSBS_OK;
}

int gsbs_debug_get_cells(gsbs_ctx* c, int64_t max_n, int32_t* cell, uint64_t* uid, int32_t* nc, int64_t* n) {
    if (!c || !n) return fail(GSBS_EINVAL, "null");
    DevCounters h{};
    CHK(read_counters(c, &h));
    std::vector<float4> p0(std::max<int32_t>(h.n_live, 1));
    std::vector<uint64_t> u(std::max<int32_t>(h.n_live, 1));
    if (h.n_live > 0) {
        HIPCHK(hipMemcpyAsync(p0.data(), c->pos0, sizeof(float4) * h.n_live, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipMemcpyAsync(u.data(), c->uid[c->cur], sizeof(uint64_t) * h.n_live, hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
    }
    for (int64_t k = 0; k < std::min<int64_t>(h.n_live, max_n); ++k) {
        uint32_t g;
        std::memcpy(&g, &p0[k].w, 4);
        const uint32_t ncell = (uint32_t)c->dbg_nc * (uint32_t)c->dbg_nc * (uint32_t)c->dbg_nc;
        if (cell) cell[k] = (int32_t)((uint32_t)(g - (uint32_t)c->dbg_cell_base) % (c->dbg_by_species ? ncell : 0xFFFFFFFFu));
        if (uid) uid[k] = u[k];
    }
    if (nc) *nc = c->dbg_nc;
    *n = h.n_live;
    return GSBS_OK;
}

}  // extern "C"
