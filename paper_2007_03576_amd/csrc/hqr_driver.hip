// Host driver and C-ABI of libhqr: multishift QR with aggressive early
// deflation on one GPU (Myllykoski, ACM TOMS 48(1), 2021).
//
// The driver is the single-GPU form of the paper's event-driven main loop
// (Sec. 3.3 "Event-driven algorithm"): the bottom unreduced block of the active segment is either
// handed to the small solver or gets an AED step; the AED outcome (number of
// deflated eigenvalues and the shift candidates) is the one value the host
// waits for in each iteration -- the analogue of acquiring the 'small AED'
// return handle.  A repeated AED is chosen when many eigenvalues deflated
// (Sec. 2.5); otherwise a multishift sweep is enqueued as rounds of
// concurrent bulge-chasing windows ('push bulges') followed by the left and
// right update products (Sec. 3.4 "Bulge chasing").  Updates that cannot feed back into the
// active block (columns right of it, rows above it, and Q) run on a second
// stream at default priority, ordered after their inputs by events, so the
// window chain and the AED -- the critical path of Sec. 3.4.1 -- never wait
// for them.
#include "hqr_common.h"
#include "../../include/hqr.h"
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

using namespace hqr;

namespace {

std::mutex g_mu;
hqr_params g_params = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0.0, 0, 0};

// Work-queue buffers of the batched form, one per (device, stream), grown on
// demand and kept until the process ends.
struct QueueBuf {
    int32_t *p = nullptr;
    int64_t cap = 0;
};
std::map<std::pair<int, void *>, QueueBuf> g_queues;

// Workspace of the backward pass, one per (device, stream), grow-only: host
// staging (pinned) for the orders, offsets and descriptors, the device
// descriptor table and the per-chunk workspace.  A call that fits the current
// capacities allocates nothing; calls on one stream are serialized by mu.
struct BwdWs {
    std::mutex mu;
    int32_t *h_n = nullptr;
    int64_t *h_off = nullptr;
    BwdDesc *h_desc = nullptr;
    int64_t hcap = 0;
    BwdDesc *d_desc = nullptr;
    int64_t dcap = 0;
    double *ws = nullptr;
    size_t wcap = 0;
};
std::map<std::pair<int, void *>, BwdWs> g_bwd;

// Launch shape of the batched global-memory grid: workgroups per CU, and the
// order above which matrices go to half of that grid only.  Per bulge
// position a workgroup touches about 176*n bytes of H and Q (n cache lines
// for three rows, three columns of H and Q); two workgroups per CU keep that
// inside the CU's share of L2 (4 MB per 32 CUs) up to about n = 360.
int g_batched_wg_per_cu = 2, g_batched_wide_n = 320;
// Per-bucket AED window and shift count of the batched form (empty: double
// shifts for every order), chosen by the package's autotuner.
BatchedTable g_btab = {0, {0}, {0}, {0}};
constexpr int NSTATS = 12;
thread_local int64_t t_stats[NSTATS];

struct Params {
    int ns, nw, nmin, nibble, kexsh;
    int64_t itmax;
    int window, gsize;
    int streams;
    int nsmall; // shifts per multishift sweep of the one-workgroup solver (2 = double shift)
    int aed_ns, aed_nw, aed_nmin; // recursive solve of large AED windows (0 = automatic)
    int defl_mode;                // 0 LAPACK-style, 1 norm-stable, 2 fixed (Sec. 5.6)
    double defl_thold;            // threshold of the fixed conditions
    int aed_mode;                 // large AED windows: 0 adaptive, 1 sequential, 2 parallel (Sec. 3.5)
    int seq_max;                  // largest window of the sequential AED
    int aed_nibble;               // nibble of the recursive solve (0 = automatic)
};

// Reading of the repeated-AED heuristic (Sec. 2.5) on this GPU: the sweep is
// skipped when an AED step deflated more than nibble % of its window.  An AED
// step is a chain of one-CU kernels while a sweep over a large block spreads
// over many CUs, so above NIBBLE_BIG_BLOCK rows the sweep is skipped only
// after a very productive AED (measured at n = 16384, prescribed spectrum:
// 14 % -> 23.7 s, 60 % -> 10.9 s, 100 % -> 10.8 s; at n = 4096, Gaussian,
// where AED deflates about 85 % of each window, 14 % and 40 % alike); for
// smaller blocks, where a sweep is a few small chase launches, LAPACK's 14 %
// (the recursive solve of 256-windows at n = 4096: 14 % 0.68 s, 25 % 0.77 s,
// 40 % 1.03 s).  An explicit nibble applies at every size.
constexpr int NIBBLE_SMALL = 14, NIBBLE_BIG = 60, NIBBLE_BIG_BLOCK = 256;

int nibble_for(const Params &P, int nh)
{
    if (P.nibble > 0) return P.nibble;
    return nh > NIBBLE_BIG_BLOCK ? NIBBLE_BIG : NIBBLE_SMALL;
}

// Reading of automatic parameters: LAPACK's documented shift-count table and
// an AED window of ns (order <= 500) or 3ns/2 above, capped where noted.
void auto_ns_nw(int nh, int &ns, int &nw)
{
    int s;
    if (nh < 30) s = 2;
    else if (nh < 60) s = 4;
    else if (nh < 150) s = 10;
    else if (nh < 590) {
        int lg = (int)std::lround(std::log2((double)nh));
        s = std::max(10, nh / std::max(lg, 1));
    } else if (nh < 3000) s = 64;
    else if (nh < 6000) s = 128;
    else s = 256;
    s &= ~1;
    ns = s;
    nw = (nh <= 500) ? s : 3 * s / 2;
}

hipError_t g_err = hipSuccess;
#define CK(x)                                                                                                 \
    do {                                                                                                       \
        hipError_t e_ = (x);                                                                                   \
        if (e_ != hipSuccess) {                                                                                \
            g_err = e_;                                                                                        \
            return -1000 - (int)e_;                                                                            \
        }                                                                                                      \
    } while (0)

// Undeflated orders of a large AED window from which the Hessenberg
// restoration runs as the blocked many-CU reduction instead of one workgroup.
constexpr int RESTORE_BLOCKED_MIN = 128;

struct Workspace {
    int dev = -1;
    hipStream_t lo = nullptr;          // deferred-update stream
    IterStatus *st_dev = nullptr;
    IterStatus *st_host = nullptr;     // pinned
    double *sh_host = nullptr;         // pinned shifts staging
    double *d_shift = nullptr;         // device shifts (re, im)
    double *ubuf = nullptr;            // ring of window factors
    int nslots = 0;
    int slot_next = 0;
    std::vector<hipEvent_t> slot_ev;   // recorded on lo after the slot's last use
    std::vector<char> slot_used;
    double *fin = nullptr;             // finalize scratch
    size_t fin_n = 0;
    std::vector<double *> wT, wV, wU;  // per recursion depth: AED window, its factor, factor^T
    std::vector<int> wcap;
    std::vector<hipEvent_t> wU_ev;     // recorded on lo after the last deferred use of wU
    std::vector<char> wU_pending;
    double *vbuf = nullptr;
    double *hws = nullptr;             // blocked Hessenberg reduction workspace
    size_t hws_n = 0;
    int *flag = nullptr;
    hipEvent_t ev_pool[64];
    int ev_next = 0;
    // update work queued on the deferred stream: one event per flush with its
    // counted flops (a ring; the adaptive AED decision pops finished entries)
    static constexpr int NPOOL = 32;
    hipEvent_t pool_ev[NPOOL];
    double pool_fl[NPOOL];
    int pool_head = 0, pool_n = 0;
    // sequential AED time model t = seq_a w^3 (seconds), refined from the
    // measured sequential AEDs
    hipEvent_t seq_t0 = nullptr, seq_t1 = nullptr;
    double seq_a = 2.5e-9;
    bool init = false;
};

Workspace g_ws[16];
// Calls on one device run one at a time: they share its workspace.
std::mutex g_ws_mu[16];

// ---- optional kernel-class timing with HIP events (measurement tools) ----
constexpr int NCLASS = 5; // 0 LDS iteration, 1 chase windows, 2 update products, 3 large-AED kernels, 4 other
constexpr int NTICK = 10;
struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;
double g_prof_ms[NCLASS], g_prof_flops[NCLASS], g_prof_bytes[NCLASS];
int64_t g_prof_n[NCLASS];
// LDS iteration kernel: wall-clock ticks of Schur solve, reordering, restoration and total, then
// bulge-chase phases, single-bulge steps, swaps, launches of the small-solve and AED kinds, and
// phases of the pipelined reordering
long long g_prof_ticks[NTICK];

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

int prof_begin(int cls, hipStream_t s)
{
    if (!g_prof_on) return -1;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    ProfRec r;
    r.cls = cls;
    r.a = prof_event();
    r.b = prof_event();
    r.flops = r.bytes = 0.0;
    hipEventRecord(r.a, s);
    g_prof.push_back(r);
    return (int)g_prof.size() - 1;
}

void prof_end(int id, hipStream_t s, double flops, double bytes)
{
    if (id < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEventRecord(g_prof[id].b, s);
    g_prof[id].flops = flops;
    g_prof[id].bytes = bytes;
}

void prof_set_flops(int id, double flops)
{
    if (id < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[id].flops = flops;
}

void prof_add_ticks(const IterStatus &S)
{
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < 4; ++i) g_prof_ticks[i] += S.tick[i];
    g_prof_ticks[4] += S.nphase;
    g_prof_ticks[5] += S.nbstep;
    g_prof_ticks[6] += S.nswap;
    g_prof_ticks[S.kind == 0 ? 7 : 8] += 1;
    g_prof_ticks[9] += S.nrphase;
}

// fold finished records into the per-class totals
void prof_collect()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof) {
        hipEventSynchronize(r.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_prof_ms[r.cls] += ms;
            g_prof_flops[r.cls] += r.flops;
            g_prof_bytes[r.cls] += r.bytes;
            g_prof_n[r.cls] += 1;
        }
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof.clear();
}

int slot_ustride() { return WMAX * WMAX; }

struct Ctx {
    Workspace *W;
    hipStream_t hi; // caller's stream: the critical path
    bool two;       // deferred updates on W->lo
    Defl dfl;       // deflation conditions
    Params P;
    int64_t *stats;
};

int ensure_ws(Workspace &W, int dev)
{
    if (W.init) return 0;
    W.dev = dev;
    CK(hipStreamCreateWithFlags(&W.lo, hipStreamNonBlocking));
    CK(hipMalloc(&W.st_dev, sizeof(IterStatus)));
    CK(hipHostMalloc(&W.st_host, sizeof(IterStatus), hipHostMallocDefault));
    CK(hipHostMalloc(&W.sh_host, sizeof(double) * 2 * 2048, hipHostMallocDefault));
    CK(hipMalloc(&W.d_shift, sizeof(double) * 2 * 2048));
    W.nslots = 512;
    CK(hipMalloc(&W.ubuf, sizeof(double) * (size_t)slot_ustride() * W.nslots));
    W.slot_ev.resize(W.nslots);
    W.slot_used.assign(W.nslots, 0);
    for (int i = 0; i < W.nslots; ++i) CK(hipEventCreateWithFlags(&W.slot_ev[i], hipEventDisableTiming));
    for (int i = 0; i < 64; ++i) CK(hipEventCreateWithFlags(&W.ev_pool[i], hipEventDisableTiming));
    for (int i = 0; i < Workspace::NPOOL; ++i) CK(hipEventCreateWithFlags(&W.pool_ev[i], hipEventDisableTiming));
    CK(hipEventCreate(&W.seq_t0));
    CK(hipEventCreate(&W.seq_t1));
    CK(hipMalloc(&W.flag, sizeof(int) * 4));
    W.init = true;
    return 0;
}

hipEvent_t next_event(Workspace &W)
{
    hipEvent_t e = W.ev_pool[W.ev_next];
    W.ev_next = (W.ev_next + 1) % 64;
    return e;
}

// A slot of the factor ring; waits (on the critical stream) until the
// deferred stream has finished with its previous contents.
int take_slot(Ctx &C)
{
    Workspace &W = *C.W;
    int s = W.slot_next;
    W.slot_next = (W.slot_next + 1) % W.nslots;
    // the deferred stream may still read this slot (from any recursion level)
    if (W.slot_used[s]) {
        hipStreamWaitEvent(C.hi, W.slot_ev[s], 0);
        W.slot_used[s] = 0;
    }
    return s;
}

double *slot_ptr(Workspace &W, int s) { return W.ubuf + (size_t)s * slot_ustride(); }

// Marks the slot as read by deferred work enqueued so far on the second stream.
void release_slot(Ctx &C, int s)
{
    if (C.two) {
        hipEventRecord(C.W->slot_ev[s], C.W->lo);
        C.W->slot_used[s] = 1;
    }
}

int ensure_depth(Workspace &W, int depth, int w)
{
    if ((int)W.wT.size() <= depth) {
        W.wT.resize(depth + 1, nullptr);
        W.wV.resize(depth + 1, nullptr);
        W.wU.resize(depth + 1, nullptr);
        W.wcap.resize(depth + 1, 0);
        size_t old = W.wU_ev.size();
        W.wU_ev.resize(depth + 1, nullptr);
        W.wU_pending.resize(depth + 1, 0);
        for (size_t d = old; d <= (size_t)depth; ++d) CK(hipEventCreateWithFlags(&W.wU_ev[d], hipEventDisableTiming));
    }
    if (W.wcap[depth] >= w) return 0;
    if (W.wT[depth]) {
        hipFree(W.wT[depth]);
        hipFree(W.wV[depth]);
        hipFree(W.wU[depth]);
    }
    int w16 = (w + 15) & ~15;
    CK(hipMalloc(&W.wT[depth], sizeof(double) * (size_t)w * w));
    CK(hipMalloc(&W.wV[depth], sizeof(double) * (size_t)w * w));
    CK(hipMalloc(&W.wU[depth], sizeof(double) * (size_t)w16 * w16));
    W.wcap[depth] = w;
    if (!W.vbuf) CK(hipMalloc(&W.vbuf, sizeof(double) * 16384));
    return 0;
}

// Matrix view: H (n x n, ld), Q (nq rows, ldq) -- transformations act on
// H's full rows/columns and on Q's columns.
struct View {
    double *H;
    int64_t ld;
    int n;
    double *Q;
    int64_t ldq;
    int nq;
};

void add_job(UpdBatch &b, double *X, int64_t ldx, int count, int K, const double *Ut, int side)
{
    if (count <= 0 || K <= 0) return;
    int K16 = (K + 15) & ~15;
    UpdJob &J = b.job[b.njobs];
    J.X = X;
    J.Ut = Ut;
    J.ldx = ldx;
    J.count = count;
    J.K = K;
    J.K16 = K16;
    J.side = side;
    J.tile = update_tile(K16, side);
    J.tiles = (count + J.tile - 1) / J.tile;
    b.first_tile[b.njobs + 1] = b.first_tile[b.njobs] + J.tiles;
    b.njobs++;
}

int flush(UpdBatch &b, hipStream_t s, Ctx &C)
{
    if (b.njobs > 0) {
        double fl = 0.0, by = 0.0;
        for (int j = 0; j < b.njobs; ++j) {
            double K = b.job[j].K, cnt = b.job[j].count;
            fl += 2.0 * K * K * cnt;
            by += 16.0 * K * cnt + 8.0 * K * K;
        }
        int pid = prof_begin(2, s);
        CK(launch_updates(b, s));
        prof_end(pid, s, fl, by);
        if (C.stats) C.stats[6]++;
        Workspace &W = *C.W;
        if (C.two && s == W.lo) {
            if (W.pool_n == Workspace::NPOOL) { // ring full: forget the oldest entry
                W.pool_head = (W.pool_head + 1) % Workspace::NPOOL;
                W.pool_n--;
            }
            const int slot = (W.pool_head + W.pool_n) % Workspace::NPOOL;
            CK(hipEventRecord(W.pool_ev[slot], s));
            W.pool_fl[slot] = fl;
            W.pool_n++;
        }
    }
    b.njobs = 0;
    b.first_tile[0] = 0;
    return 0;
}

UpdBatch make_batch()
{
    UpdBatch b;
    b.njobs = 0;
    b.first_tile[0] = 0;
    return b;
}

// Apply the factor of a transformed diagonal block [kw, kw+m) of the active
// block [ktop, kbot] to the rest of the view.  Parts inside the active block
// run on the critical stream; the rest (and Q) on the deferred stream.
int apply_factor(Ctx &C, const View &V, int ktop, int kbot, int kw, int m, const double *Ut)
{
    UpdBatch hiL = make_batch(), hiR = make_batch(), loL = make_batch(), loR = make_batch();
    int c0 = kw + m; // first column right of the block
    int ncol_in = std::max(0, std::min(kbot, V.n - 1) - c0 + 1);
    int ncol_out = V.n - c0 - ncol_in;
    int nrow_in = std::max(0, kw - ktop);
    int nrow_out = kw - nrow_in;
    if (!C.two) {
        add_job(hiL, V.H + kw + (int64_t)c0 * V.ld, V.ld, V.n - c0, m, Ut, 1);
        add_job(hiR, V.H + (int64_t)kw * V.ld, V.ld, kw, m, Ut, 0);
        if (V.Q) add_job(hiR, V.Q + (int64_t)kw * V.ldq, V.ldq, V.nq, m, Ut, 0);
        if (flush(hiL, C.hi, C)) return g_err ? -1000 - (int)g_err : -1;
        if (flush(hiR, C.hi, C)) return -1;
        return 0;
    }
    add_job(hiL, V.H + kw + (int64_t)c0 * V.ld, V.ld, ncol_in, m, Ut, 1);
    add_job(hiR, V.H + ktop + (int64_t)kw * V.ld, V.ld, nrow_in, m, Ut, 0);
    add_job(loL, V.H + kw + (int64_t)(c0 + ncol_in) * V.ld, V.ld, ncol_out, m, Ut, 1);
    add_job(loR, V.H + (int64_t)kw * V.ld, V.ld, nrow_out, m, Ut, 0);
    if (V.Q) add_job(loR, V.Q + (int64_t)kw * V.ldq, V.ldq, V.nq, m, Ut, 0);
    // critical updates
    if (flush(hiL, C.hi, C)) return -1;
    if (flush(hiR, C.hi, C)) return -1;
    // deferred updates: after the factor exists and after the critical
    // updates (the deferred regions never overlap the active block, but the
    // left/right products of one factor share no data, so only the factor
    // itself orders them)
    if (loL.njobs + loR.njobs > 0) {
        hipEvent_t e = next_event(*C.W);
        hipEventRecord(e, C.hi);
        hipStreamWaitEvent(C.W->lo, e, 0);
        if (flush(loL, C.W->lo, C)) return -1;
        if (flush(loR, C.W->lo, C)) return -1;
    }
    return 0;
}

int read_status(Ctx &C, int ncand)
{
    Workspace &W = *C.W;
    size_t head = offsetof(IterStatus, cr);
    CK(hipMemcpyAsync(W.st_host, W.st_dev, head, hipMemcpyDeviceToHost, C.hi));
    if (ncand > 0) {
        ncand = std::min(ncand, MAXCAND);
        CK(hipMemcpyAsync(W.st_host->cr, W.st_dev->cr, sizeof(double) * ncand, hipMemcpyDeviceToHost, C.hi));
        CK(hipMemcpyAsync(W.st_host->ci, W.st_dev->ci, sizeof(double) * ncand, hipMemcpyDeviceToHost, C.hi));
    }
    CK(hipStreamSynchronize(C.hi));
    if (C.stats) C.stats[5]++;
    return 0;
}

// --------------------------------------------------------------------------
// multishift sweep

int sweep(Ctx &C, const View &V, int ktop, int kbot, int nsh, const double *sr, const double *si)
{
    Workspace &W = *C.W;
    int nb = nsh / 2;
    if (nb <= 0) return 0;
    for (int i = 0; i < nsh; ++i) {
        W.sh_host[i] = sr[i];
        W.sh_host[2048 + i] = si[i];
    }
    CK(hipMemcpyAsync(W.d_shift, W.sh_host, sizeof(double) * nsh, hipMemcpyHostToDevice, C.hi));
    CK(hipMemcpyAsync(W.d_shift + 2048, W.sh_host + 2048, sizeof(double) * nsh, hipMemcpyHostToDevice, C.hi));
    int w = std::min(C.P.window, WMAX);
    int g = std::min(nb, std::min(C.P.gsize, GMAX));
    // the window must hold the group chain plus room to move
    while (g > 1 && 3 * g + 2 > w - 8) --g;
    int ngroups = (nb + g - 1) / g;
    struct Grp {
        int nb, p0, soff;
        bool started, done;
    };
    std::vector<Grp> G(ngroups);
    for (int i = 0; i < ngroups; ++i) {
        G[i].nb = std::min(g, nb - i * g);
        G[i].p0 = ktop - 1;
        G[i].soff = 2 * i * g;
        G[i].started = false;
        G[i].done = false;
    }
    int remaining = ngroups;
    int guard = 0;
    while (remaining > 0) {
        if (++guard > 100000) return -99;
        ChaseRound R;
        R.nwin = 0;
        R.ktop = ktop;
        R.kbot = kbot;
        int lower_a = INT32_MAX; // top of the window of the next lower group this round
        for (int gi = 0; gi < ngroups && R.nwin < MAXWIN; ++gi) {
            Grp &gr = G[gi];
            if (gr.done) continue;
            int a;
            if (!gr.started) {
                a = ktop;
            } else {
                a = gr.p0 - 3 * (gr.nb - 1);
            }
            int wa = std::min(w, kbot - a + 1);
            if (a + wa > lower_a) wa = lower_a - a;
            bool final_w = (a + wa - 1 >= kbot);
            int kend = final_w ? kbot - 2 : a + wa - 5;
            int top_next = gr.p0 - 3 * (gr.nb - 1);
            int nsteps;
            if (final_w)
                nsteps = (kbot - 2) - top_next + 1;
            else
                nsteps = kend - gr.p0 + 1;
            bool ok = wa >= 4 && nsteps > 0 && (final_w || wa >= 3 * gr.nb + 2);
            if (!ok) {
                if (!gr.started) break; // later groups cannot start either
                lower_a = std::min(lower_a, a);
                continue;
            }
            ChaseWin &cw = R.w[R.nwin];
            cw.a = a;
            cw.wa = wa;
            cw.p0 = gr.p0;
            cw.nsteps = nsteps;
            cw.kend = kend;
            cw.nb = gr.nb;
            cw.shift_off = gr.soff;
            cw.slot = take_slot(C);
            // vigilant deflation (Sec. 3.2, 'push bulges'): only the windows of
            // the last chain of the sweep scan the subdiagonal, behind its top
            // bulge, where the entries are final for this sweep
            int tpos0 = gr.p0 - 3 * (gr.nb - 1);
            cw.vig_lo = std::max(ktop, tpos0);
            cw.vig_hi = std::min(kend, tpos0 + nsteps - 1);
            if (cw.vig_hi - cw.vig_lo + 1 > WMAX) cw.vig_lo = cw.vig_hi - WMAX + 1;
            if (gi != ngroups - 1) {
                cw.vig_lo = 1;
                cw.vig_hi = 0;
            }
            R.nwin++;
            gr.started = true;
            gr.p0 += nsteps;
            if (final_w) {
                gr.done = true;
                --remaining;
            }
            lower_a = a;
        }
        if (R.nwin == 0) return -98;
        int pid = prof_begin(1, C.hi);
        CK(launch_chase(V.H, V.ld, R, W.d_shift, W.d_shift + 2048, C.dfl, W.ubuf, slot_ustride(), C.hi));
        {
            double fl = 0.0, by = 0.0;
            for (int i = 0; i < R.nwin; ++i) {
                // direct-reflector flops inside the window: about 11 per touched
                // entry, 3 rows + 3 columns of A and 3 columns of U per reflector
                double wa = R.w[i].wa;
                fl += 12.0 * (2.0 * wa + 5.0) * R.w[i].nb * R.w[i].nsteps;
                by += 2.0 * 8.0 * wa * wa + 8.0 * wa * wa;
            }
            prof_end(pid, C.hi, fl, by);
        }
        if (C.stats) {
            C.stats[6]++;
            C.stats[7] += R.nwin;
        }
        // update products: all left products first (disjoint rows), then all
        // right products (disjoint columns)
        UpdBatch hiL = make_batch(), hiR = make_batch(), loL = make_batch(), loR = make_batch();
        for (int i = 0; i < R.nwin; ++i) {
            const ChaseWin &cw = R.w[i];
            const double *Ut = slot_ptr(W, cw.slot);
            int c0 = cw.a + cw.wa;
            if (!C.two) {
                add_job(hiL, V.H + cw.a + (int64_t)c0 * V.ld, V.ld, V.n - c0, cw.wa, Ut, 1);
                add_job(hiR, V.H + (int64_t)cw.a * V.ld, V.ld, cw.a, cw.wa, Ut, 0);
                if (V.Q) add_job(hiR, V.Q + (int64_t)cw.a * V.ldq, V.ldq, V.nq, cw.wa, Ut, 0);
            } else {
                int ncol_in = std::max(0, kbot - c0 + 1);
                add_job(hiL, V.H + cw.a + (int64_t)c0 * V.ld, V.ld, ncol_in, cw.wa, Ut, 1);
                add_job(loL, V.H + cw.a + (int64_t)(c0 + ncol_in) * V.ld, V.ld, V.n - c0 - ncol_in, cw.wa, Ut,
                        1);
                int nrow_in = std::max(0, cw.a - ktop);
                add_job(hiR, V.H + ktop + (int64_t)cw.a * V.ld, V.ld, nrow_in, cw.wa, Ut, 0);
                add_job(loR, V.H + (int64_t)cw.a * V.ld, V.ld, cw.a - nrow_in, cw.wa, Ut, 0);
                if (V.Q) add_job(loR, V.Q + (int64_t)cw.a * V.ldq, V.ldq, V.nq, cw.wa, Ut, 0);
            }
        }
        if (flush(hiL, C.hi, C)) return -1;
        if (flush(hiR, C.hi, C)) return -1;
        if (C.two) {
            hipEvent_t e = next_event(W);
            hipEventRecord(e, C.hi);
            hipStreamWaitEvent(W.lo, e, 0);
            if (flush(loL, W.lo, C)) return -1;
            if (flush(loR, W.lo, C)) return -1;
            for (int i = 0; i < R.nwin; ++i) release_slot(C, R.w[i].slot);
        }
    }
    return 0;
}

// --------------------------------------------------------------------------
// driver

int run(Ctx &C, const View &V, int ilo, int ihi, const Params &P, int depth, int *info_out);

// Optional progress report of long solves (environment HQR_PROGRESS=1): one
// line on stderr per top-level AED step, at most one every two seconds.
void progress_line(int ilo, int kbot, int nd)
{
    static std::chrono::steady_clock::time_point last;
    const char *e = std::getenv("HQR_PROGRESS");
    if (!(e && e[0] == '1')) return;
    const auto now = std::chrono::steady_clock::now();
    if (now - last < std::chrono::seconds(2)) return;
    last = now;
    std::fprintf(stderr, "hqr: AED step deflated %d, %d rows left above row %d\n", nd, kbot - ilo + 1, ilo);
    std::fflush(stderr);
}

// AED step with a window larger than the LDS solver: recursive Schur form of
// a copy of the window, corner deflation, Hessenberg restoration.
// Update flops still queued on the deferred stream (finished flushes are
// dropped by querying their events; no synchronization).
double pool_pending(Workspace &W)
{
    while (W.pool_n > 0 && hipEventQuery(W.pool_ev[W.pool_head]) == hipSuccess) {
        W.pool_head = (W.pool_head + 1) % Workspace::NPOOL;
        W.pool_n--;
    }
    double fl = 0.0;
    for (int i = 0; i < W.pool_n; ++i) fl += W.pool_fl[(W.pool_head + i) % Workspace::NPOOL];
    return fl;
}

// Rate assumed for queued update work in the adaptive AED decision: the
// update kernels' measured throughput on this GPU is 6..13 TFLOP/s.
constexpr double POOL_RATE = 10e12;

int big_aed(Ctx &C, const View &V, int ktop, int kbot, int w, int depth, int &nd, int &ns, int &ncand)
{
    Workspace &W = *C.W;
    if (ensure_depth(W, depth, w)) return -1;
    int kwtop = kbot - w + 1;
    double s = 0.0;
    if (kwtop > ktop) {
        CK(hipMemcpyAsync(&W.st_host->beta, V.H + kwtop + (int64_t)(kwtop - 1) * V.ld, sizeof(double),
                          hipMemcpyDeviceToHost, C.hi));
        CK(hipStreamSynchronize(C.hi));
        s = W.st_host->beta;
    }
    double *T = W.wT[depth], *Vw = W.wV[depth], *Ut = W.wU[depth];
    CK(launch_window_copy(V.H, V.ld, kwtop, w, T, w, Vw, w, C.hi));
    // Sequential or parallel AED (Sec. 3.5, "Adaptive approach").  The
    // sequential AED runs on one workgroup, so it is preferred when it is
    // predicted to finish while the deferred stream is still busy with queued
    // updates that it overlaps; otherwise the window is solved in parallel.
    bool seq = false;
    if (w <= C.P.seq_max) {
        if (C.P.aed_mode == 1) {
            seq = true;
        } else if (C.P.aed_mode == 0 && C.two) {
            const double t_seq = W.seq_a * (double)w * (double)w * (double)w;
            seq = t_seq <= pool_pending(W) / POOL_RATE;
        }
    }
    int bot = w;
    if (seq) {
        const int nwb = std::min(64, std::max(24, w / 4)), nsb = std::min(64, std::max(2, w / 4)) & ~1;
        int pids = prof_begin(3, C.hi);
        CK(hipEventRecord(W.seq_t0, C.hi));
        CK(launch_seq_aed(T, w, Vw, s, C.dfl, nwb, nsb, W.st_dev, C.hi));
        CK(hipEventRecord(W.seq_t1, C.hi));
        prof_end(pids, C.hi, 10.0 * (double)w * w * w, 0.0);
        if (C.stats) C.stats[10]++;
        if (read_status(C, 0)) return -1;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, W.seq_t0, W.seq_t1) == hipSuccess && ms > 0.0f)
            W.seq_a = 0.5 * W.seq_a + 0.5 * (1e-3 * ms / ((double)w * w * w));
        if (W.st_host->info > 0) { // the window did not converge: discard it
            nd = 0;
            ns = w;
            CK(launch_block_eigs(T, w, w, W.st_dev->cr, W.st_dev->ci, C.hi));
            if (read_status(C, w)) return -1;
            ncand = w;
            return 0;
        }
        bot = W.st_host->ns;
    } else {
        if (C.stats) C.stats[11]++;
        // Reading for the recursive solve of the window: AED windows of w/4
        // (48..96, within the one-workgroup solver) and as many shifts per sweep
        // as such a window delivers (at most w/4).  Measured at n = 16384 (AED
        // windows of 1024): nw/4 shifts 48.8 s per solve, 64 shifts 29.7 s, nw
        // shifts 27.3 s; at n = 4096 (windows of 256) no difference.
        Params Pi = C.P;
        Pi.nw = std::min(std::max(w / 4, 48), MMAX);
        Pi.ns = std::max(2, Pi.nw & ~1);
        if (C.P.aed_nw > 0) Pi.nw = C.P.aed_nw;
        if (C.P.aed_ns > 0) Pi.ns = C.P.aed_ns;
        if (C.P.aed_nmin > 0) Pi.nmin = C.P.aed_nmin;
        if (C.P.aed_nibble > 0) Pi.nibble = C.P.aed_nibble;
        Pi.ns = std::min(Pi.ns, std::max(2, (w / 4) & ~1));
        Pi.itmax = C.P.itmax;
        View Vi{T, w, w, Vw, w, w};
        Ctx Ci = C;
        Ci.two = false; // the window is small; keep its updates in order on one stream
        int info = 0;
        int rc = run(Ci, Vi, 0, w - 1, Pi, depth + 1, &info);
        if (rc) return rc;
        if (info > 0) {
            nd = 0;
            ns = w;
            CK(launch_block_eigs(T, w, w, W.st_dev->cr, W.st_dev->ci, C.hi));
            if (read_status(C, w)) return -1;
            ncand = w;
            return 0;
        }
        // Deflation check of the whole window (Sec. 3.5 "Parallel aggressive
        // early deflation"): deflation windows of order <= 96 move up from the
        // bottom corner.  Each examines its unchecked candidates bottom-up (the
        // failures of the window below it, at its bottom, count as failed) and
        // leaves all failures at its top; the next window ends at the bottommost
        // failure.  When the failures fill more than half of a window (and at
        // most two thirds), a chain of reordering windows carries them to the top
        // of the AED window and the next deflation window starts at the next
        // unevaluated candidate; with more failures the rest of the window counts
        // as undeflated (few of its candidates would deflate).  The
        // transformation of each window updates the window rows to its right,
        // the rows above it and V.  A rejected swap halts the check (the greedy
        // rule): everything above the deflated bottom then counts as undeflated.
        int nfail = 0, ntop = 0;
        auto window = [&](int wbot, int wd, int nforced, int reorder, int &c0, int &wdd, int &halted,
                          int &nsr) -> int {
            int slc = take_slot(C);
            double *Utc = slot_ptr(W, slc); // used on the critical stream only
            int pidc = prof_begin(3, C.hi);
            CK(launch_corner_deflate(T, w, wbot, wd, Vw, w, s, C.dfl, Utc, W.st_dev, nforced, reorder, C.hi));
            prof_end(pidc, C.hi, 0.0, 0.0);
            if (C.stats) C.stats[reorder ? 9 : 8]++;
            if (read_status(C, 0)) return -1;
            c0 = W.st_host->kwtop;
            wdd = W.st_host->nw;
            halted = W.st_host->info;
            nsr = W.st_host->ns; // undeflated leading rows of the AED window
            UpdBatch b = make_batch();
            add_job(b, T + (int64_t)c0 * w, w, c0, wdd, Utc, 0);
            add_job(b, T + c0 + (int64_t)wbot * w, w, w - wbot, wdd, Utc, 1);
            add_job(b, Vw + (int64_t)c0 * w, w, w, wdd, Utc, 0);
            if (flush(b, C.hi, C)) return -1;
            return 0;
        };
        for (;;) {
            const int wd = std::min(bot - ntop, MMAX); // the failures already at the top stay out
            if (wd <= nfail) break;
            int c0, wdd, halted, nsr;
            const int rw = window(bot, wd, nfail, 0, c0, wdd, halted, nsr);
            if (rw) return rw;
            const int nf = nsr - c0; // failures now at [c0, nsr), deflated below
            bot = nsr;
            if (halted || c0 <= ntop) break;
            if (2 * nf <= wdd) {
                nfail = nf;
                continue;
            }
            // a reordering window advances by its order minus the failures it
            // carries: beyond two thirds of a window the rest is left unevaluated
            if (3 * nf > 2 * wdd) break;
            // reordering chain: failures [fb - nf, fb) up to [ntop, ntop + nf)
            int fb = nsr;
            bool moved = true;
            while (fb - nf > ntop) {
                const int wr = std::min(fb - ntop, MMAX);
                if (wr <= nf + 1) {
                    moved = false; // no room to pass a block
                    break;
                }
                int c0r, wdr, haltedr, nsrr;
                const int rr = window(fb, wr, nf, 1, c0r, wdr, haltedr, nsrr);
                if (rr) return rr;
                if (haltedr || c0r + nf >= fb) {
                    moved = false;
                    break;
                }
                fb = c0r + nf;
            }
            if (!moved) break;
            ntop += nf;
            nfail = 0;
        }
    }
    ns = bot;
    nd = w - bot;
    CK(launch_block_eigs(T, w, ns, W.st_dev->cr, W.st_dev->ci, C.hi));
    ncand = ns;
    if (nd > 0) {
        double beta = 0.0;
        if (ns > 1 && s != 0.0) {
            int pidr = prof_begin(3, C.hi);
            if (ns >= RESTORE_BLOCKED_MIN) {
                // many-CU blocked reduction (panels, GEMV, FP64-MFMA updates)
                const size_t need = hess_ws_doubles(ns, w - ns, w);
                if (W.hws_n < need) {
                    if (W.hws) {
                        CK(hipStreamSynchronize(C.hi));
                        CK(hipFree(W.hws));
                    }
                    W.hws = nullptr;
                    W.hws_n = 0;
                    CK(hipMalloc(&W.hws, sizeof(double) * need));
                    W.hws_n = need;
                }
                CK(restore_blocked(T, w, w, ns, Vw, w, w, s, W.hws, &W.st_dev->beta, C.hi));
            } else {
                CK(launch_restore(T, w, w, ns, Vw, w, w, s, W.vbuf, W.st_dev, C.hi));
            }
            prof_end(pidr, C.hi, 10.0 / 3.0 * (double)ns * ns * ns + 4.0 * (double)w * ns * ns, 0.0);
            CK(hipMemcpyAsync(&W.st_host->beta, &W.st_dev->beta, sizeof(double), hipMemcpyDeviceToHost, C.hi));
        } else if (ns >= 1) {
            CK(hipMemcpyAsync(&W.st_host->beta, Vw, sizeof(double), hipMemcpyDeviceToHost, C.hi));
        }
        if (read_status(C, ncand)) return -1;
        if (ns > 1 && s != 0.0) beta = W.st_host->beta;
        else if (ns >= 1) beta = s * W.st_host->beta;
        // copy the window back (zeros below the subdiagonal) and set the new subdiagonal
        CK(hipMemcpy2DAsync(V.H + kwtop + (int64_t)kwtop * V.ld, V.ld * sizeof(double), T, w * sizeof(double),
                            w * sizeof(double), w, hipMemcpyDeviceToDevice, C.hi));
        CK(launch_zero_lower(V.H + kwtop + (int64_t)kwtop * V.ld, V.ld, w, C.hi));
        if (kwtop > ktop) {
            W.st_host->beta = beta;
            CK(hipMemcpyAsync(V.H + kwtop + (int64_t)(kwtop - 1) * V.ld, &W.st_host->beta, sizeof(double),
                              hipMemcpyHostToDevice, C.hi));
        }
        int w16 = (w + 15) & ~15;
        if (C.two && W.wU_pending[depth]) CK(hipStreamWaitEvent(C.hi, W.wU_ev[depth], 0));
        CK(launch_transpose_pad(Vw, w, w, Ut, w16, C.hi));
        int rc2 = apply_factor(C, V, ktop, kbot, kwtop, w, Ut);
        if (rc2) return rc2;
        if (C.two) {
            CK(hipEventRecord(W.wU_ev[depth], W.lo));
            W.wU_pending[depth] = 1;
        }
        // the host value for the subdiagonal must stay alive until the copy ran
        CK(hipStreamSynchronize(C.hi));
    } else {
        if (read_status(C, ncand)) return -1;
    }
    return 0;
}

int run(Ctx &C, const View &V, int ilo, int ihi, const Params &P, int depth, int *info_out)
{
    Workspace &W = *C.W;
    IterStatus &S = *W.st_host;
    int kbot = ihi;
    int64_t it = 0;
    int ndfl = 1;
    std::vector<double> sr(2048), si(2048), cr, ci;
    *info_out = 0;
    while (kbot >= ilo) {
        int ktop, nd = 0, ns = 0, ncand = 0, wwin = 0;
        bool aed = false;
        int nwp = std::min(P.nw, MMAX);
        if (P.nw <= MMAX) {
            int sl = take_slot(C);
            double *Ut = slot_ptr(W, sl);
            int pid = prof_begin(0, C.hi);
            CK(launch_iter(V.H, V.ld, V.n, ilo, kbot, P.nw, P.nmin, C.dfl, P.itmax, Ut, W.st_dev, C.hi, P.nsmall));
            prof_end(pid, C.hi, 0.0, 0.0);
            if (C.stats) C.stats[6]++;
            if (read_status(C, nwp)) return -1;
            prof_set_flops(pid, S.beta);
            prof_add_ticks(S);
            ktop = S.ktop;
            if (S.kind == 0) {
                // the block was written back with the factor of the steps it
                // took, converged or not: propagate it so that H = Q T Q^T holds
                const int finfo = S.info;
                if (C.stats) C.stats[4]++;
                int rc = apply_factor(C, V, ktop, kbot, S.kwtop, S.nw, Ut);
                release_slot(C, sl);
                if (rc) return rc;
                if (finfo > 0) {
                    *info_out = finfo;
                    return 0;
                }
                kbot = ktop - 1;
                ndfl = 1;
                continue;
            }
            aed = true;
            nd = S.nd;
            ns = S.ns;
            ncand = S.ncand;
            wwin = S.nw;
            if (S.changed) {
                int rc = apply_factor(C, V, ktop, kbot, S.kwtop, S.nw, Ut);
                if (rc) return rc;
            }
            release_slot(C, sl);
        } else {
            CK(launch_find_block(V.H, V.ld, ilo, kbot, C.dfl, W.st_dev, C.hi));
            if (read_status(C, 0)) return -1;
            ktop = S.ktop;
            int nh = kbot - ktop + 1;
            int wv = std::min(P.nw, nh);
            if (nh <= P.nmin || wv <= MMAX) {
                int sl = take_slot(C);
                double *Ut = slot_ptr(W, sl);
                int pid = prof_begin(0, C.hi);
                CK(launch_iter(V.H, V.ld, V.n, ilo, kbot, wv, P.nmin, C.dfl, P.itmax, Ut, W.st_dev, C.hi, P.nsmall));
                prof_end(pid, C.hi, 0.0, 0.0);
                if (read_status(C, MMAX)) return -1;
                prof_set_flops(pid, S.beta);
                prof_add_ticks(S);
                if (S.kind == 0) {
                    const int finfo = S.info;
                    if (C.stats) C.stats[4]++;
                    int rc = apply_factor(C, V, ktop, kbot, S.kwtop, S.nw, Ut);
                    release_slot(C, sl);
                    if (rc) return rc;
                    if (finfo > 0) {
                        *info_out = finfo;
                        return 0;
                    }
                    kbot = ktop - 1;
                    ndfl = 1;
                    continue;
                }
                nd = S.nd;
                ns = S.ns;
                ncand = S.ncand;
                wwin = S.nw;
                if (S.changed) {
                    int rc = apply_factor(C, V, ktop, kbot, S.kwtop, S.nw, Ut);
                    if (rc) return rc;
                }
                release_slot(C, sl);
            } else {
                int rc = big_aed(C, V, ktop, kbot, wv, depth, nd, ns, ncand);
                if (rc) return rc;
                wwin = wv;
            }
            aed = true;
        }
        (void)aed;
        if (++it > P.itmax) {
            *info_out = kbot + 1;
            return 0;
        }
        if (C.stats && depth == 0) {
            C.stats[0]++;
            C.stats[3] += nd;
        }
        if (depth == 0) progress_line(ilo, kbot - nd, nd);
        cr.assign(S.cr, S.cr + ncand);
        ci.assign(S.ci, S.ci + ncand);
        const int nh_aed = kbot - ktop + 1; // the active block the AED step saw
        kbot -= nd;
        ndfl = (nd > 0) ? 1 : ndfl + 1;
        if (nd > 0 && 100 * nd > nibble_for(P, nh_aed) * wwin) continue;
        if (kbot - ktop + 1 <= P.nmin) continue;
        int nsh = 0;
        if (ndfl % P.kexsh == 0) {
            // Reading: exceptional shifts from the trailing subdiagonal
            int want = P.ns;
            if (want > kbot - ktop - 1) want = (kbot - ktop - 1) & ~1;
            int cnt = std::min(want, kbot - ktop);
            int lo_row = std::max(ktop, kbot - std::min(cnt + 2, MAXCAND - 1));
            int rows = kbot - lo_row + 1;
            // the diagonal and subdiagonal entries of rows lo_row..kbot: both
            // are vectors of stride ld + 1, fetched by one strided copy each
            // into the pinned candidate arrays (their values were taken above)
            double *diag = S.cr, *sub = S.ci;
            const size_t pitch = (size_t)(V.ld + 1) * sizeof(double);
            CK(hipMemcpy2DAsync(diag, sizeof(double), V.H + lo_row + (int64_t)lo_row * V.ld, pitch, sizeof(double),
                                rows, hipMemcpyDeviceToHost, C.hi));
            const int s0 = (lo_row == 0) ? 1 : 0; // row 0 has no subdiagonal entry
            if (s0) sub[0] = 0.0;
            if (rows > s0)
                CK(hipMemcpy2DAsync(sub + s0, sizeof(double), V.H + (lo_row + s0) + (int64_t)(lo_row + s0 - 1) * V.ld,
                                    pitch, sizeof(double), rows - s0, hipMemcpyDeviceToHost, C.hi));
            CK(hipStreamSynchronize(C.hi));
            for (int i = kbot; i >= ktop + 2 && nsh + 2 <= want; i -= 2) {
                int li = i - lo_row;
                if (li - 1 < 0) break;
                double ss = std::fabs(sub[li]) + std::fabs(sub[li - 1]);
                double a = 0.75 * ss + diag[li];
                double w2 = ss * std::sqrt(0.4375);
                sr[nsh] = a;
                si[nsh] = w2;
                sr[nsh + 1] = a;
                si[nsh + 1] = -w2;
                nsh += 2;
            }
        } else {
            // Reading: bottommost candidates, conjugate pairs together, real
            // shifts paired in order, an odd real left over dropped.
            int nc = ncand;
            int want = std::min(P.ns, nc);
            int start = nc - want;
            if (start > 0 && start < nc && ci[start] < 0.0) start++;
            double rr[2];
            int nr = 0;
            for (int i = nc - 1; i >= start; --i) {
                if (ci[i] != 0.0) {
                    if (ci[i] < 0.0 && i - 1 >= start) {
                        sr[nsh] = cr[i - 1];
                        si[nsh] = ci[i - 1];
                        sr[nsh + 1] = cr[i];
                        si[nsh + 1] = ci[i];
                        nsh += 2;
                        --i;
                    }
                } else {
                    rr[nr++] = cr[i];
                    if (nr == 2) {
                        sr[nsh] = rr[0];
                        si[nsh] = 0.0;
                        sr[nsh + 1] = rr[1];
                        si[nsh + 1] = 0.0;
                        nsh += 2;
                        nr = 0;
                    }
                }
            }
            if (nsh < 2 || (nd > 0 && nsh < P.ns / 2)) continue;
        }
        if (nsh < 2) continue;
        int rc = sweep(C, V, ktop, kbot, nsh, sr.data(), si.data());
        if (rc) return rc;
        if (C.stats && depth == 0) {
            C.stats[1]++;
            C.stats[2] += nsh;
        }
    }
    return 0;
}

// Deflation mode 0 (LAPACK-style), 1 (norm-stable) or 2 (fixed, with a finite
// threshold >= 0).
bool defl_ok(const hqr_params *p)
{
    if (p->aed_mode < 0 || p->aed_mode > 2 || p->aed_seq_max < 0) return false;
    if (p->defl_mode == 0 || p->defl_mode == 1) return true;
    return p->defl_mode == 2 && p->defl_thold >= 0.0 && std::isfinite(p->defl_thold);
}

Params resolve(const hqr_params *pp, int n)
{
    hqr_params p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        p = g_params;
    }
    if (pp) p = *pp;
    Params P;
    auto_ns_nw(n, P.ns, P.nw);
    if (p.ns > 0) P.ns = p.ns & ~1;
    if (p.nw > 0) P.nw = p.nw;
    if (P.ns < 2) P.ns = 2;
    P.nmin = p.nmin > 0 ? p.nmin : 75;
    P.nmin = std::max(12, std::min(P.nmin, MMAX));
    P.nibble = p.nibble > 0 ? p.nibble : 0; // 0: nibble_for's size rule
    P.kexsh = p.kexsh > 0 ? p.kexsh : 6;
    P.itmax = p.itmax > 0 ? p.itmax : 30 * (int64_t)std::max(10, n);
    P.window = p.window > 0 ? std::min(p.window, WMAX) : WMAX;
    P.gsize = p.bulges_per_window > 0 ? std::min(p.bulges_per_window, GMAX) : GMAX;
    P.streams = p.streams > 0 ? p.streams : 2;
    P.nsmall = p.small_shifts > 0 ? std::min(p.small_shifts, 16) & ~1 : 2;
    P.aed_ns = p.aed_ns > 0 ? std::max(2, p.aed_ns & ~1) : 0;
    P.aed_nw = p.aed_nw > 0 ? std::max(4, std::min(p.aed_nw, MMAX)) : 0;
    P.aed_nmin = p.aed_nmin > 0 ? std::max(12, std::min(p.aed_nmin, MMAX)) : 0;
    if (P.nw < 2) P.nw = 2;
    P.nw = std::min(P.nw, MAX_UPDATE_K);
    P.defl_mode = p.defl_mode;
    P.defl_thold = p.defl_thold;
    P.aed_mode = p.aed_mode;
    P.seq_max = p.aed_seq_max > 0 ? std::min(p.aed_seq_max, MAX_UPDATE_K) : 512;
    P.aed_nibble = p.aed_nibble > 0 ? p.aed_nibble : 0;
    return P;
}

} // namespace

extern "C" {

int hqr_set_params(const hqr_params *p)
{
    if (!p) return -1;
    if (p->ns < 0 || p->nw < 0 || p->nmin < 0 || p->window < 0 || !defl_ok(p)) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    g_params = *p;
    return 0;
}

int hqr_get_params(hqr_params *p)
{
    if (!p) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    *p = g_params;
    return 0;
}

int hqr_schur_ex(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi, void *stream,
                 const hqr_params *pp)
{
    for (int i = 0; i < NSTATS; ++i) t_stats[i] = 0;
    if (n < 0) return -3;
    if (n == 0) return 0;
    if (!H) return -1;
    if (ld < std::max<int64_t>(1, n)) return -4;
    if (!wr) return -5;
    if (!wi) return -6;
    if (n > (int64_t)INT32_MAX / 2) return -3;
    if (pp && !defl_ok(pp)) return -8;
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16) return -1000;
    Workspace &W = g_ws[dev];
    std::lock_guard<std::mutex> lk(g_ws_mu[dev]);
    int e = ensure_ws(W, dev);
    if (e) return e;
    Params P = resolve(pp, (int)n);
    Ctx C;
    C.W = &W;
    C.hi = (hipStream_t)stream;
    C.two = P.streams >= 2;
    C.dfl.smlnum = DBL_MIN * ((double)n / DBL_EPSILON);
    C.dfl.thr = (P.defl_mode == 2) ? P.defl_thold : -1.0;
    C.P = P;
    C.stats = t_stats;
    if (W.fin_n < (size_t)n) {
        if (W.fin) {
            CK(hipDeviceSynchronize()); // an earlier call may still finish on another stream
            CK(hipFree(W.fin));
        }
        W.fin = nullptr;
        W.fin_n = 0;
        CK(hipMalloc(&W.fin, sizeof(double) * 8 * (size_t)n));
        W.fin_n = n;
    }
    // argument check on the device: non-finite entries of the Hessenberg part
    CK(hipMemsetAsync(W.flag, 0, sizeof(int), C.hi));
    CK(launch_check_finite(H, ld, (int)n, W.flag, C.hi));
    CK(hipMemcpyAsync(&W.st_host->pad, W.flag, sizeof(int), hipMemcpyDeviceToHost, C.hi));
    if (P.defl_mode == 1) {
        // norm-stable conditions: u ||H||_F of the input (an orthogonal
        // similarity keeps the norm, so one value serves the whole solve)
        CK(launch_hess_fro(H, ld, (int)n, W.fin, &W.st_dev->beta, C.hi));
        CK(hipMemcpyAsync(&W.st_host->beta, &W.st_dev->beta, sizeof(double), hipMemcpyDeviceToHost, C.hi));
    }
    CK(hipStreamSynchronize(C.hi));
    if (W.st_host->pad) return -1;
    if (P.defl_mode == 1) C.dfl.thr = DBL_EPSILON * W.st_host->beta;
    CK(launch_zero_lower(H, ld, (int)n, C.hi));
    View V{H, ld, (int)n, Q, ld, Q ? (int)n : 0};
    int info = 0;
    int rc = run(C, V, 0, (int)n - 1, P, 0, &info);
    if (rc) {
        hipStreamSynchronize(W.lo);
        return rc;
    }
    // join the deferred stream, then standardize and extract eigenvalues
    if (C.two) {
        hipEvent_t ev = next_event(W);
        CK(hipEventRecord(ev, W.lo));
        CK(hipStreamWaitEvent(C.hi, ev, 0));
    }
    int pidf = prof_begin(4, C.hi);
    CK(launch_finalize_ws(H, ld, (int)n, info > 0 ? info : 0, Q, wr, wi, W.fin, C.hi));
    prof_end(pidf, C.hi, 0.0, 0.0);
    CK(hipStreamSynchronize(C.hi));
    for (int i = 0; i < W.nslots; ++i) W.slot_used[i] = 0;
    return info;
}

int hqr_schur(double *H, double *Q, int64_t n, int64_t ld, double *wr, double *wi, void *stream)
{
    return hqr_schur_ex(H, Q, n, ld, wr, wi, stream, nullptr);
}

int hqr_hessenberg(double *A, double *Q, int64_t n, int64_t ld, void *stream)
{
    if (n < 0) return -3;
    if (n == 0) return 0;
    if (!A) return -1;
    if (ld < std::max<int64_t>(1, n)) return -4;
    if (n > (int64_t)INT32_MAX / 2) return -3;
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16) return -1000;
    Workspace &W = g_ws[dev];
    std::lock_guard<std::mutex> lk(g_ws_mu[dev]);
    int e = ensure_ws(W, dev);
    if (e) return e;
    hipStream_t st = (hipStream_t)stream;
    // argument check on the device: non-finite entries
    CK(hipMemsetAsync(W.flag, 0, sizeof(int), st));
    CK(launch_check_finite_full(A, ld, (int)n, W.flag, st));
    CK(hipMemcpyAsync(&W.st_host->pad, W.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (W.st_host->pad) return -1;
    const size_t need = hess_ws_doubles((int)n, 0, Q ? (int)n : 0);
    if (W.hws_n < need) {
        if (W.hws) CK(hipFree(W.hws)); // the stream was synchronized above
        W.hws = nullptr;
        W.hws_n = 0;
        CK(hipMalloc(&W.hws, sizeof(double) * need));
        W.hws_n = need;
    }
    CK(hess_reduce(A, ld, (int)n, 0, Q, ld, Q ? (int)n : 0, W.hws, st));
    CK(launch_zero_lower(A, ld, (int)n, st));
    CK(hipStreamSynchronize(st)); // the workspace is reused by the next call
    return 0;
}

int hqr_last_stats(int64_t *stats, int len)
{
    if (!stats || len <= 0) return 0;
    int m = std::min(len, NSTATS);
    for (int i = 0; i < m; ++i) stats[i] = t_stats[i];
    return m;
}

int hqr_profile_enable(int on)
{
    g_prof_on = on != 0;
    return 0;
}

int hqr_profile_reset(void)
{
    prof_collect();
    for (int c = 0; c < NCLASS; ++c) {
        g_prof_ms[c] = g_prof_flops[c] = g_prof_bytes[c] = 0.0;
        g_prof_n[c] = 0;
    }
    for (int i = 0; i < NTICK; ++i) g_prof_ticks[i] = 0;
    return 0;
}

int hqr_profile_ticks(int64_t *ticks, int len)
{
    if (!ticks || len <= 0) return -1;
    int m = std::min(len, NTICK);
    for (int i = 0; i < m; ++i) ticks[i] = g_prof_ticks[i];
    return m;
}

int hqr_profile_read(double *ms, int64_t *launches, double *flops, double *bytes, int nclass)
{
    if (!ms || !launches || !flops || !bytes || nclass <= 0) return -1;
    prof_collect();
    int m = std::min(nclass, NCLASS);
    for (int c = 0; c < m; ++c) {
        ms[c] = g_prof_ms[c];
        launches[c] = g_prof_n[c];
        flops[c] = g_prof_flops[c];
        bytes[c] = g_prof_bytes[c];
    }
    return m;
}

int hqr_finalize(void)
{
    free_update_ws();
    for (auto &W : g_ws) {
        if (!W.init) continue;
        hipSetDevice(W.dev);
        hipDeviceSynchronize();
        for (auto e : W.slot_ev) hipEventDestroy(e);
        for (int i = 0; i < 64; ++i) hipEventDestroy(W.ev_pool[i]);
        for (int i = 0; i < Workspace::NPOOL; ++i) hipEventDestroy(W.pool_ev[i]);
        hipEventDestroy(W.seq_t0);
        hipEventDestroy(W.seq_t1);
        hipStreamDestroy(W.lo);
        hipFree(W.st_dev);
        hipHostFree(W.st_host);
        hipHostFree(W.sh_host);
        hipFree(W.d_shift);
        hipFree(W.ubuf);
        hipFree(W.fin);
        hipFree(W.vbuf);
        hipFree(W.hws);
        hipFree(W.flag);
        for (auto e : W.wU_ev) hipEventDestroy(e);
        for (size_t d = 0; d < W.wT.size(); ++d) {
            hipFree(W.wT[d]);
            hipFree(W.wV[d]);
            hipFree(W.wU[d]);
        }
        W = Workspace();
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_queues) {
        hipSetDevice(kv.first.first);
        hipDeviceSynchronize();
        hipFree(kv.second.p);
    }
    g_queues.clear();
    for (auto &kv : g_bwd) {
        hipSetDevice(kv.first.first);
        hipDeviceSynchronize();
        BwdWs &B = kv.second;
        hipHostFree(B.h_n);
        hipHostFree(B.h_off);
        hipHostFree(B.h_desc);
        hipFree(B.d_desc);
        hipFree(B.ws);
    }
    g_bwd.clear();
    return 0;
}

int hqr_qz_batched(double *H, double *T, double *Q, double *Z, const int64_t *offsets, const int32_t *n,
                   int32_t batch, double *alphar, double *alphai, double *beta, const int64_t *eig_offsets,
                   int32_t *info, void *stream)
{
    if (batch < 0) return -7;
    if (batch == 0) return 0;
    if (!H) return -1;
    if (!T) return -2;
    if (!offsets) return -5;
    if (!n) return -6;
    if (!alphar) return -8;
    if (!alphai) return -9;
    if (!beta) return -10;
    if (!eig_offsets) return -11;
    if (!info) return -12;
    CK(launch_qz_batched(H, T, Q, Z, offsets, n, batch, alphar, alphai, beta, eig_offsets, info,
                         (hipStream_t)stream));
    return 0;
}

int hqr_schur_batched(double *H, double *Q, const int64_t *offsets, const int32_t *n, int32_t batch, double *wr,
                      double *wi, const int64_t *eig_offsets, int32_t *info, void *stream)
{
    if (batch < 0) return -5;
    if (batch == 0) return 0;
    if (!H) return -1;
    if (!offsets) return -3;
    if (!n) return -4;
    if (!wr) return -6;
    if (!wi) return -7;
    if (!eig_offsets) return -8;
    if (!info) return -9;
    int32_t *queue = nullptr;
    int wg_per_cu, wide_n;
    BatchedTable tab;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        wg_per_cu = g_batched_wg_per_cu;
        wide_n = g_batched_wide_n;
        tab = g_btab;
        int dev = 0;
        CK(hipGetDevice(&dev));
        QueueBuf &qb = g_queues[std::make_pair(dev, stream)];
        const int64_t need = (int64_t)batch + QHDR;
        if (qb.cap < need) {
            if (qb.p) {
                CK(hipStreamSynchronize((hipStream_t)stream)); // earlier calls on this stream still read it
                CK(hipFree(qb.p));
            }
            qb.p = nullptr;
            qb.cap = 0;
            CK(hipMalloc((void **)&qb.p, need * sizeof(int32_t)));
            qb.cap = need;
        }
        queue = qb.p;
    }
    CK(launch_batched(H, Q, offsets, n, batch, wr, wi, eig_offsets, info, queue, wg_per_cu, wide_n, tab,
                      (hipStream_t)stream));
    return 0;
}

} // extern "C"

// Work queue of hqr_schur_batched_noalloc: a fixed device array (each GPU
// holds its own copy for the life of the process), so that entry point never
// allocates.  Host code reaches it only through the address that
// hipGetSymbolAddress returns on each device.
constexpr int64_t NOALLOC_MAX_BATCH = (int64_t)1 << 20;
static __device__ __align__(256) int32_t scratch[QHDR + NOALLOC_MAX_BATCH];

namespace {
std::mutex g_scratch_mu;
int32_t *g_scratch_ptr[16] = {nullptr};
} // namespace

extern "C" {

int hqr_schur_batched_noalloc(double *H, double *Q, const int64_t *offsets, const int32_t *n, int32_t batch,
                              double *wr, double *wi, const int64_t *eig_offsets, int32_t *info, void *stream)
{
    if (batch < 0 || (int64_t)batch > NOALLOC_MAX_BATCH) return -5;
    if (batch == 0) return 0;
    if (!H) return -1;
    if (!offsets) return -3;
    if (!n) return -4;
    if (!wr) return -6;
    if (!wi) return -7;
    if (!eig_offsets) return -8;
    if (!info) return -9;
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 16) return -1000;
    int32_t *queue;
    int wg_per_cu, wide_n;
    BatchedTable tab;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            CK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            g_scratch_ptr[dev] = static_cast<int32_t *>(ptr);
        }
        queue = g_scratch_ptr[dev];
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        wg_per_cu = g_batched_wg_per_cu;
        wide_n = g_batched_wide_n;
        tab = g_btab;
    }
    // the sort kernel writes every queue head and position it uses, so the
    // array needs no clearing between calls
    CK(launch_batched(H, Q, offsets, n, batch, wr, wi, eig_offsets, info, queue, wg_per_cu, wide_n, tab,
                      (hipStream_t)stream));
    return 0;
}

int hqr_set_batched_launch(int32_t wg_per_cu, int32_t wide_n)
{
    if (wg_per_cu < 1 || wg_per_cu > 8) return -1;
    if (wide_n < MMAX || wide_n > 4095) return -2;
    std::lock_guard<std::mutex> lk(g_mu);
    g_batched_wg_per_cu = wg_per_cu;
    g_batched_wide_n = wide_n;
    return 0;
}

int hqr_set_batched_table(int32_t nb, const int32_t *upper, const int32_t *nw, const int32_t *ns)
{
    if (nb < 0 || nb > MAXBUCKET) return -1;
    if (nb > 0 && (!upper || !nw || !ns)) return -2;
    BatchedTable t = {0, {0}, {0}, {0}};
    for (int i = 0; i < nb; ++i) {
        if (upper[i] < 1 || (i > 0 && upper[i] <= upper[i - 1])) return -2;
        if (nw[i] != 0 && (nw[i] < 8 || nw[i] > BWIN)) return -3;
        if (ns[i] < 0 || (ns[i] & 1) || (nw[i] != 0 && ns[i] < 2) || ns[i] > BWIN) return -4;
        t.upper[i] = upper[i];
        t.nw[i] = nw[i];
        t.ns[i] = ns[i];
    }
    t.nb = nb;
    std::lock_guard<std::mutex> lk(g_mu);
    g_btab = t;
    return 0;
}

int hqr_get_batched_table(int32_t *nb, int32_t *upper, int32_t *nw, int32_t *ns)
{
    if (!nb || !upper || !nw || !ns) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    *nb = g_btab.nb;
    for (int i = 0; i < MAXBUCKET; ++i) {
        upper[i] = g_btab.upper[i];
        nw[i] = g_btab.nw[i];
        ns[i] = g_btab.ns[i];
    }
    return 0;
}

int hqr_get_batched_launch(int32_t *wg_per_cu, int32_t *wide_n)
{
    if (!wg_per_cu || !wide_n) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    *wg_per_cu = g_batched_wg_per_cu;
    *wide_n = g_batched_wide_n;
    return 0;
}


int hqr_eigenvectors(const double *T, const double *Q, int64_t n, int64_t ld, const double *wr, const double *wi,
                     double *X, int64_t ldx, void *stream)
{
    if (!T) return -1;
    if (!Q) return -2;
    if (n < 0 || n > 8192) return -3;
    if (ld < std::max<int64_t>(1, n)) return -4;
    if (!wr) return -5;
    if (!wi) return -6;
    if (!X) return -7;
    if (ldx < std::max<int64_t>(1, n)) return -8;
    if (n == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    CK(hipGetDevice(&dev));
    BwdWs *B;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        B = &g_bwd[std::make_pair(dev, stream)];
    }
    std::lock_guard<std::mutex> call_lk(B->mu);
    const size_t nn = (size_t)n * n;
    const size_t need = 10 * nn + 1 + 2 * nn; // backward layout, then packed copies of T and Q
    if (B->wcap < need || B->dcap < 1) {
        CK(hipStreamSynchronize(st)); // earlier calls on this stream may still use the buffers
        if (B->wcap < need) {
            if (B->ws) CK(hipFree(B->ws));
            B->ws = nullptr;
            B->wcap = 0;
            CK(hipMalloc(&B->ws, sizeof(double) * need));
            B->wcap = need;
        }
        if (B->dcap < 1) {
            if (B->d_desc) CK(hipFree(B->d_desc));
            B->d_desc = nullptr;
            B->dcap = 0;
            CK(hipMalloc(&B->d_desc, sizeof(BwdDesc)));
            B->dcap = 1;
        }
    }
    double *Tp = B->ws + 10 * nn + 1, *Qp = Tp + nn;
    CK(hipMemcpy2DAsync(Tp, n * sizeof(double), T, ld * sizeof(double), n * sizeof(double), n,
                        hipMemcpyDeviceToDevice, st));
    CK(hipMemcpy2DAsync(Qp, n * sizeof(double), Q, ld * sizeof(double), n * sizeof(double), n,
                        hipMemcpyDeviceToDevice, st));
    BwdDesc d{0, 0, 0, (int)n, 0};
    CK(hipMemcpyAsync(B->d_desc, &d, sizeof(BwdDesc), hipMemcpyHostToDevice, st));
    CK(launch_eigenvectors(Tp, Qp, B->d_desc, (int)n, wr, wi, B->ws, X, ldx, st));
    CK(hipStreamSynchronize(st)); // the descriptor lives on the host stack
    return 0;
}

int hqr_eig_backward_batched(const double *T, const double *Q, const int64_t *offsets, const int32_t *n,
                             int32_t batch, const double *wr, const double *wi, const double *gwr,
                             const double *gwi, double *dH, int32_t hess_mask, void *stream)
{
    if (!T) return -1;
    if (!Q) return -2;
    if (!offsets) return -3;
    if (!n) return -4;
    if (batch < 0) return -5;
    if (!wr) return -6;
    if (!wi) return -7;
    if (!gwr) return -8;
    if (!gwi) return -9;
    if (!dH) return -10;
    if (batch == 0) return 0;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    CK(hipGetDevice(&dev));
    BwdWs *B;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        B = &g_bwd[std::make_pair(dev, stream)];
    }
    std::lock_guard<std::mutex> call_lk(B->mu);
    // the orders and offsets are read on the host to plan the chunks; the
    // stream is synchronized here, so every earlier call on it (and its reads
    // of the staging buffers) has finished
    if (B->hcap < batch) {
        if (B->h_n) CK(hipHostFree(B->h_n));
        if (B->h_off) CK(hipHostFree(B->h_off));
        if (B->h_desc) CK(hipHostFree(B->h_desc));
        B->h_n = nullptr;
        B->h_off = nullptr;
        B->h_desc = nullptr;
        B->hcap = 0;
        CK(hipHostMalloc(&B->h_n, sizeof(int32_t) * (size_t)batch, hipHostMallocDefault));
        CK(hipHostMalloc(&B->h_off, sizeof(int64_t) * (size_t)batch, hipHostMallocDefault));
        CK(hipHostMalloc(&B->h_desc, sizeof(BwdDesc) * (size_t)batch, hipHostMallocDefault));
        B->hcap = batch;
    }
    CK(hipMemcpyAsync(B->h_n, n, sizeof(int32_t) * (size_t)batch, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(B->h_off, offsets, sizeof(int64_t) * (size_t)batch, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    // descriptors and chunks: a chunk's workspace stays within 2 GiB unless a
    // single matrix needs more
    const size_t cap_doubles = ((size_t)1 << 31) / sizeof(double);
    int64_t eo = 0;
    size_t need_max = 0, run = 0;
    for (int32_t b = 0; b < batch; ++b) {
        const int32_t nb_ = B->h_n[b];
        if (nb_ < 0 || nb_ > 8192) return -4;
        if (B->h_off[b] < 0) return -3;
        const size_t wsz = 10 * (size_t)nb_ * nb_ + 1;
        if (run > 0 && run + wsz > cap_doubles) run = 0;
        BwdDesc &d = B->h_desc[b];
        d.toff = B->h_off[b];
        d.eoff = eo;
        d.woff = (int64_t)run;
        d.n = nb_;
        d.pad = 0;
        run += wsz;
        need_max = std::max(need_max, run);
        eo += nb_;
    }
    if (B->dcap < batch) {
        if (B->d_desc) CK(hipFree(B->d_desc));
        B->d_desc = nullptr;
        B->dcap = 0;
        CK(hipMalloc(&B->d_desc, sizeof(BwdDesc) * (size_t)batch));
        B->dcap = batch;
    }
    if (B->wcap < need_max) {
        if (B->ws) CK(hipFree(B->ws));
        B->ws = nullptr;
        B->wcap = 0;
        CK(hipMalloc(&B->ws, sizeof(double) * need_max));
        B->wcap = need_max;
    }
    CK(hipMemcpyAsync(B->d_desc, B->h_desc, sizeof(BwdDesc) * (size_t)batch, hipMemcpyHostToDevice, st));
    int32_t b0 = 0;
    while (b0 < batch) {
        int32_t b1 = b0 + 1;
        int nmax = B->h_n[b0];
        while (b1 < batch && B->h_desc[b1].woff != 0) {
            nmax = std::max(nmax, (int)B->h_n[b1]);
            ++b1;
        }
        CK(launch_eig_backward_chunk(T, Q, B->d_desc + b0, b1 - b0, nmax, wr, wi, gwr, gwi, dH, hess_mask,
                                     B->ws, st));
        b0 = b1;
    }
    return 0;
}

} // extern "C"
