// fca_api.hip -- host runtime of libfca: the C ABI declared in include/fca.h.
//
// A context owns, in device memory: the mixtures in the EM layout
// y_int[f][m][n] (complex, row pitch npad = N rounded up to 64), the powers
// v[j][f][n] (same pitch), the per-frequency state P (M x M complex FP64,
// stride 64 entries), Lambda (stride 8), log|det P|^2 and status flags, the
// initial values for fca_reset, and the per-iteration log-likelihood of every
// (mixture, frequency). The EM problems are sorted into launch groups of equal
// (M, frames per thread), largest N first, and each group is one launch of
// the per-frequency EM kernel per chunk of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <limits>
#include <vector>

#include "fca.h"
#include "fca_internal.h"

using namespace fca;

namespace {

constexpr int kLChunk = 128;  // iterations per EM launch (log-likelihood buffer depth)

struct MixInfo {
    int M, N, npad, fpt;
    int64_t y_base;   // complex elements into y
    int64_t v_base;   // reals into v (and v_init)
    int64_t R_base;   // complex128 elements into R_init
    int64_t out_R;    // complex128 elements into a batch R_out
    int64_t out_v;    // reals into a batch v_out
    int64_t out_x;    // complex elements into a batch x_out
    int pid0;         // first problem index (b * F)
    bool has_v0;
    bool R_default;   // R_init holds the plain start (no launch needed to restore it)
};

// A launch group: problems of equal M and frames-per-thread class (fpt for
// kEmThreads threads, 0 = streamed), consecutive in the problem table. nt and
// run_fpt are the launch shape used (kEmThreads and fpt unless tuned).
struct Group {
    int M, fpt, first, count, max_n;
    int nt = kEmThreads, run_fpt = 0;
};

constexpr int kMaxSide = 3;  // extra streams for concurrent launch groups

thread_local std::string g_init_error;

}  // namespace

struct fca_ctx {
    int B = 0, F = 0;
    bool fp64 = true;
    hipStream_t stream = nullptr;
    size_t esz = 16, rsz = 8;
    std::vector<MixInfo> mix;
    std::vector<Group> groups;
    int nprob = 0;
    int64_t v_alt = 0;  // element offset of the second power buffer (streaming problems)

    void* y = nullptr;
    void* v = nullptr;
    void* v_init = nullptr;
    double2* R_init = nullptr;
    double2* P = nullptr;
    double2* Pinv = nullptr;  // P^-1 per problem (for the separation)
    // the stored start's basis (P, Lambda, log|det P|^2 of theta^(0)); with
    // v_init it makes a reset a handful of whole-buffer copies
    double2* P0 = nullptr;
    double* lam0 = nullptr;
    double* logdet0 = nullptr;
    double* lam = nullptr;
    double* logdet = nullptr;
    int* flags = nullptr;
    double* ll = nullptr;
    double* ll_tot = nullptr;
    double* ll_host = nullptr;  // pinned
    int* flag_sum = nullptr;       // device: OR of the flags, first NOT_PD, first NONFINITE, their iterations
    int* flag_sum_host = nullptr;  // pinned copy
    double* fsum = nullptr;
    double2* R_stage = nullptr;
    EmProblem* probs = nullptr;
    int64_t* x_off = nullptr;
    std::vector<int> flags_host;
    int64_t v_tot = 0;  // reals in one power buffer (v, v_init)

    // Launch tables: every problem (probs, groups; used by fca_separate) and
    // the problems of active mixtures only (probs_act, groups_act; used by the
    // EM calls while some mixture is inactive), rebuilt lazily.
    std::vector<EmProblem> table;
    MaskCovMix* mask_mix = nullptr;       // device table of fca_set_mask_covariances (B entries)
    MaskCovMix* mask_mix_host = nullptr;  // pinned staging of it
    EmProblem* table_act = nullptr;  // pinned host staging of probs_act (nprob entries)
    int* inactive_host = nullptr;    // pinned host staging of inactive_dev (B entries)
    hipEvent_t table_ev = nullptr;   // the last upload from table_act or inactive_host
    int* inactive_dev = nullptr;     // indices of the inactive mixtures at the last table rebuild
    int n_inactive = 0;
    EmProblem* probs_act = nullptr;
    std::vector<Group> groups_act;
    std::vector<char> active;
    bool all_active = true;
    bool act_dirty = false;

    // concurrent launch groups: side streams forked from and joined to the
    // context's stream with events (captured as parallel graph branches)
    hipStream_t side[kMaxSide] = {nullptr, nullptr, nullptr};
    int nside = 0;
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kMaxSide] = {nullptr, nullptr, nullptr};

    // captured step (fca_graph_capture / fca_graph_launch)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t shape_version = 0;  // bumped when activity or launch shapes change
    int64_t graph_version = -1;

    // per-problem log-likelihood rows left in ll by the last EM call (its
    // final chunk) and the mixtures that call ran (fca_loglik_per_freq)
    int last_rows = 0;
    std::vector<char> last_active;
    int graph_rows = 0;  // the same for the captured step

    bool broken = false;
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double em_ms = 0.0;
    int64_t em_launches = 0;
    std::string err;
};

namespace {

void set_err(fca_ctx* c, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_init_error = buf;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // an unregistered host pointer is not an error here
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.isManaged;
}

#define FCA_HIP(c, call)                                                                 \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_err((c), "%s failed: %s", #call, hipGetErrorString(e_));                 \
            if (c) (c)->broken = true;                                                   \
            return FCA_E_DEVICE;                                                         \
        }                                                                                \
    } while (0)

template <typename P>
fca_status dev_alloc(fca_ctx* c, P** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (hipMalloc(reinterpret_cast<void**>(p), bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_err(c, "hipMalloc of %zu bytes failed", bytes);
        *p = nullptr;
        return FCA_E_NOMEM;
    }
    return FCA_OK;
}

void free_ctx_memory(fca_ctx* c) {
    void* dev[] = {c->y, c->v, c->v_init, c->R_init, c->P, c->Pinv, c->lam, c->logdet, c->flags, c->ll,
                   c->ll_tot, c->fsum, c->R_stage, c->probs, c->x_off, c->probs_act, c->flag_sum,
                   c->P0, c->lam0, c->logdet0, c->mask_mix, c->inactive_dev};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (c->ll_host) (void)hipHostFree(c->ll_host);
    if (c->flag_sum_host) (void)hipHostFree(c->flag_sum_host);
    if (c->table_act) (void)hipHostFree(c->table_act);
    if (c->inactive_host) (void)hipHostFree(c->inactive_host);
    if (c->mask_mix_host) (void)hipHostFree(c->mask_mix_host);
    if (c->table_ev) (void)hipEventDestroy(c->table_ev);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (int i = 0; i < kMaxSide; ++i) {
        if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
        if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
}

// Frames per thread of the resident EM kernel, or 0 (streaming kernel) when
// the frames do not fit in registers.
int frames_per_thread(int N) {
    if (N > kMaxFrames) return 0;
    int fpt = 1;
    while (fpt * kEmThreads < N) fpt *= 2;
    return fpt;
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

fca_status validate(const fca_problem* p, int b, const fca_problem* p0) {
    if (!p) { set_err(nullptr, "problem %d is NULL", b); return FCA_E_ARG; }
    if (p->M < 1 || p->M > kMaxM) { set_err(nullptr, "problem %d: M=%d outside 1..%d", b, p->M, kMaxM); return FCA_E_ARG; }
    if (p->F < 1) { set_err(nullptr, "problem %d: F=%d < 1", b, p->F); return FCA_E_ARG; }
    if (p->N < 1 || p->N > kMaxFramesStream) {
        set_err(nullptr, "problem %d: N=%d outside 1..%d", b, p->N, kMaxFramesStream);
        return FCA_E_ARG;
    }
    if (p->prec != FCA_FP64 && p->prec != FCA_FP32_BULK) { set_err(nullptr, "problem %d: bad prec %d", b, p->prec); return FCA_E_ARG; }
    if (!p->y) { set_err(nullptr, "problem %d: y is NULL", b); return FCA_E_ARG; }
    if (p->y_stride_f < 0 || p->y_stride_n < 0 || p->y_stride_m < 0) {
        set_err(nullptr, "problem %d: negative y stride", b);
        return FCA_E_ARG;
    }
    if (p0 && (p->F != p0->F || p->prec != p0->prec || p->stream != p0->stream)) {
        set_err(nullptr, "problem %d: F, prec and stream must match problem 0", b);
        return FCA_E_ARG;
    }
    return FCA_OK;
}

// The stored basis of mixture b: the FP64 GEVD of (R1^(0), R2^(0)) read from
// R (R_init of the mixture unless a staged copy is given) into P0, lam0,
// logdet0; status bits into flags. Enqueued only.
fca_status compute_basis(fca_ctx* c, int b, const double2* R, hipStream_t s) {
    const MixInfo& mi = c->mix[b];
    const int64_t mm = (int64_t)mi.M * mi.M;
    const double2* R1 = R ? R : c->R_init + mi.R_base;
    const double2* R2 = R1 + (int64_t)c->F * mm;
    FCA_HIP(c, launch_gevd(mi.M, c->F, R1, R2, mm, mm, c->P0 + (int64_t)mi.pid0 * kMaxM * kMaxM,
                           kMaxM * kMaxM, c->lam0 + (int64_t)mi.pid0 * kMaxM, kMaxM,
                           c->logdet0 + mi.pid0, c->flags + mi.pid0, s));
    return FCA_OK;
}

// The stored start (Algorithm 1, step 1) of mixture b: v^(0) in v_init (the
// plain start computed from y, unless a caller's v0 is stored there) and the
// basis (compute_basis). Enqueued only.
fca_status compute_start(fca_ctx* c, int b, const double2* R, hipStream_t s) {
    const MixInfo& mi = c->mix[b];
    if (!mi.has_v0) {
        const void* yb = static_cast<char*>(c->y) + mi.y_base * c->esz;
        double* fs = c->fsum + (int64_t)b * (c->F + 1);
        FCA_HIP(c, launch_power_sums(c->fp64, yb, mi.M, c->F, mi.N, mi.npad, fs, s));
        FCA_HIP(c, launch_default_v(c->fp64, yb, fs, mi.M, c->F, mi.N, mi.npad,
                                    static_cast<char*>(c->v_init) + mi.v_base * c->rsz, s));
    }
    return compute_basis(c, b, R, s);
}

// Copies of the stored start into the working state for problems
// [p0, p0 + np) whose powers lie at [v0, v0 + nv) reals, and zero flags:
// one launch (no memset or copy nodes when captured). Enqueued only.
fca_status restore_range(fca_ctx* c, int64_t p0, int64_t np, int64_t v0, int64_t nv, hipStream_t s) {
    auto w = [](const void* p) { return static_cast<const uint32_t*>(p); };
    auto wd = [](void* p) { return static_cast<uint32_t*>(p); };
    const int64_t vw = (int64_t)c->rsz / 4;  // words per real
    WordSegs g{};
    g.src[0] = w(static_cast<const char*>(c->v_init) + v0 * c->rsz);
    g.dst[0] = wd(static_cast<char*>(c->v) + v0 * c->rsz);
    g.end[0] = nv * vw;
    g.src[1] = w(c->P0 + p0 * kMaxM * kMaxM);
    g.dst[1] = wd(c->P + p0 * kMaxM * kMaxM);
    g.end[1] = g.end[0] + np * kMaxM * kMaxM * 4;
    g.src[2] = w(c->lam0 + p0 * kMaxM);
    g.dst[2] = wd(c->lam + p0 * kMaxM);
    g.end[2] = g.end[1] + np * kMaxM * 2;
    g.src[3] = w(c->logdet0 + p0);
    g.dst[3] = wd(c->logdet + p0);
    g.end[3] = g.end[2] + np * 2;
    g.src[4] = nullptr;
    g.dst[4] = wd(c->flags + p0);
    g.end[4] = g.end[3] + np;
    FCA_HIP(c, launch_multi_copy(g, s));
    return FCA_OK;
}

// The working state of mixture b (v, P, Lambda, log|det P|^2, flags) back to
// its stored start. Enqueued only.
fca_status restore_start(fca_ctx* c, int b, hipStream_t s) {
    const MixInfo& mi = c->mix[b];
    return restore_range(c, mi.pid0, c->F, mi.v_base, 2ll * c->F * mi.npad, s);
}

// The working state of every mixture back to its stored start. Enqueued only.
fca_status restore_all(fca_ctx* c, hipStream_t s) {
    return restore_range(c, 0, c->nprob, 0, c->v_tot, s);
}

// The stored initial powers, allocated on first use. In FP32 contexts the
// buffer starts as ones, so that the padding frames of a mixture whose
// start is written frame by frame (fca_set_learned_starts) hold 1 as the EM
// kernels expect; fca_set_start and fca_init write whole rows.
fca_status ensure_v_init(fca_ctx* c) {
    if (c->v_init) return FCA_OK;
    fca_status st = dev_alloc(c, &c->v_init, c->v_tot * c->rsz);
    if (st != FCA_OK) return st;
    if (!c->fp64) FCA_HIP(c, launch_fill_u32(c->v_init, 0x3F800000u, c->v_tot, c->stream));  // 1.0f
    return FCA_OK;
}

// Waits for the stream and reports the first frequency of mixtures
// [b0, b1) whose initial eigendecomposition failed; on success clears their
// flags (the sweep-limit bit of the initial eigendecomposition is not kept).
fca_status check_initial_flags(fca_ctx* c, int b0, int b1) {
    const hipStream_t s = c->stream;
    const int p0 = b0 * c->F, cnt = (b1 - b0) * c->F;
    FCA_HIP(c, hipMemcpyAsync(c->flags_host.data() + p0, c->flags + p0, sizeof(int) * cnt,
                              hipMemcpyDeviceToHost, s));
    FCA_HIP(c, hipStreamSynchronize(s));
    for (int i = p0; i < p0 + cnt; ++i) {
        if (c->flags_host[i] & kFreezeMask) {
            set_err(c, "initial R2 (or R1) not positive definite at mixture %d, frequency %d",
                    i / c->F, i % c->F);
            return FCA_E_NOT_PD;
        }
    }
    FCA_HIP(c, launch_fill_u32(c->flags + p0, 0u, cnt, s));
    FCA_HIP(c, hipStreamSynchronize(s));
    return FCA_OK;
}

// Every mixture back to its stored start (Algorithm 1, step 1), all active;
// waits for the stream.
fca_status do_reset(fca_ctx* c) {
    fca_status st = restore_all(c, c->stream);
    if (st != FCA_OK) return st;
    if (!c->all_active || c->act_dirty) c->shape_version += 1;
    std::fill(c->active.begin(), c->active.end(), 1);
    c->all_active = true;
    c->act_dirty = false;
    c->n_inactive = 0;
    FCA_HIP(c, hipStreamSynchronize(c->stream));
    return FCA_OK;
}

// Launch tables of the active mixtures (the full tables filtered, group
// order kept), uploaded when the set of active mixtures changed.
fca_status refresh_active(fca_ctx* c) {
    if (!c->act_dirty) return FCA_OK;
    c->act_dirty = false;
    c->shape_version += 1;
    c->all_active = std::all_of(c->active.begin(), c->active.end(), [](char a) { return a != 0; });
    c->n_inactive = 0;
    if (c->all_active) return FCA_OK;
    FCA_HIP(c, hipEventSynchronize(c->table_ev));  // the previous upload has read the staging buffers
    c->groups_act.clear();
    int n = 0;
    for (const Group& g : c->groups) {
        Group ga = g;
        ga.first = n;
        ga.count = 0;
        ga.max_n = 0;
        for (int i = g.first; i < g.first + g.count; ++i) {
            const EmProblem& e = c->table[i];
            if (!c->active[e.pid / c->F]) continue;
            c->table_act[n++] = e;
            ga.count += 1;
            ga.max_n = std::max(ga.max_n, (int)e.n);
        }
        if (ga.count) c->groups_act.push_back(ga);
    }
    if (n)
        FCA_HIP(c, hipMemcpyAsync(c->probs_act, c->table_act, (size_t)n * sizeof(EmProblem), hipMemcpyHostToDevice,
                                  c->stream));
    for (int b = 0; b < c->B; ++b)
        if (!c->active[b]) c->inactive_host[c->n_inactive++] = b;
    FCA_HIP(c, hipMemcpyAsync(c->inactive_dev, c->inactive_host, (size_t)c->n_inactive * sizeof(int),
                              hipMemcpyHostToDevice, c->stream));
    FCA_HIP(c, hipEventRecord(c->table_ev, c->stream));
    return FCA_OK;
}

// Waits for the stream; FCA_E_NOT_PD (first such problem named) if any
// problem lost positive definiteness, else FCA_E_NONFINITE if any produced a
// non-finite value. The flags are summarised on the device (three ints
// cross to the host).
fca_status check_flags(fca_ctx* c) {
    const hipStream_t s = c->stream;
    FCA_HIP(c, launch_flag_summary(c->flags, c->nprob, c->flag_sum, s));
    FCA_HIP(c, hipMemcpyAsync(c->flag_sum_host, c->flag_sum, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
    FCA_HIP(c, hipStreamSynchronize(s));
    const int np = c->flag_sum_host[1], nf = c->flag_sum_host[2];
    if (np < c->nprob) {
        set_err(c, "mixture %d, frequency %d lost positive definiteness in iteration %d of the call", np / c->F,
                np % c->F, c->flag_sum_host[3]);
        return FCA_E_NOT_PD;
    }
    if (nf < c->nprob) {
        set_err(c, "mixture %d, frequency %d produced a non-finite value in iteration %d of the call", nf / c->F,
                nf % c->F, c->flag_sum_host[4]);
        return FCA_E_NONFINITE;
    }
    return FCA_OK;
}

fca_status init_impl(const fca_problem* probs, int32_t B, fca_ctx** out) {
    const fca_problem& p0 = probs[0];
    for (int b = 0; b < B; ++b) {
        fca_status st = validate(&probs[b], b, b ? &p0 : nullptr);
        if (st != FCA_OK) return st;
    }
    fca_ctx* c = new (std::nothrow) fca_ctx();
    if (!c) { set_err(nullptr, "out of host memory"); return FCA_E_NOMEM; }
    c->B = B;
    c->F = p0.F;
    c->fp64 = (p0.prec == FCA_FP64);
    c->stream = static_cast<hipStream_t>(p0.stream);
    c->esz = c->fp64 ? 16 : 8;
    c->rsz = c->fp64 ? 8 : 4;
    c->nprob = B * c->F;
    c->flags_host.assign(c->nprob, 0);

    int64_t y_tot = 0, v_tot = 0, R_tot = 0, oR = 0, ov = 0, ox = 0;
    int maxM = 1;
    bool any_v0 = false;
    c->mix.resize(B);
    for (int b = 0; b < B; ++b) {
        MixInfo& mi = c->mix[b];
        mi.M = probs[b].M;
        mi.N = probs[b].N;
        mi.npad = (int)round_up(mi.N, 64);
        mi.fpt = frames_per_thread(mi.N);
        mi.y_base = y_tot;
        mi.v_base = v_tot;
        mi.R_base = R_tot;
        mi.out_R = oR;
        mi.out_v = ov;
        mi.out_x = ox;
        mi.pid0 = b * c->F;
        mi.has_v0 = probs[b].v0 != nullptr;
        any_v0 = any_v0 || mi.has_v0;
        maxM = std::max(maxM, mi.M);
        y_tot += (int64_t)c->F * mi.M * mi.npad;
        v_tot += 2LL * c->F * mi.npad;
        R_tot += 2LL * c->F * mi.M * mi.M;
        oR += 2LL * c->F * mi.M * mi.M;
        ov += 2LL * c->F * mi.N;
        ox += 2LL * c->F * mi.N * mi.M;
    }

    fca_status st = FCA_OK;
#define FCA_TRY(x)                                     \
    do {                                               \
        st = (x);                                      \
        if (st != FCA_OK) {                            \
            g_init_error = c->err.empty() ? g_init_error : c->err; \
            free_ctx_memory(c);                        \
            delete c;                                  \
            return st;                                 \
        }                                              \
    } while (0)

    FCA_TRY(dev_alloc(c, &c->y, y_tot * c->esz));
    bool any_stream = false;
    for (const MixInfo& mi : c->mix) any_stream = any_stream || mi.fpt == 0;
    // the second power buffer of the streaming kernel is always there, so any
    // group can be switched to streaming (fca_set_launch_shape, fca_autotune)
    (void)any_stream;
    c->v_alt = v_tot;
    c->v_tot = v_tot;
    c->active.assign(B, 1);
    FCA_TRY(dev_alloc(c, &c->v, 2 * v_tot * c->rsz));
    (void)any_v0;
    FCA_TRY(ensure_v_init(c));  // holds every mixture's stored start
    FCA_TRY(dev_alloc(c, &c->R_init, R_tot * sizeof(double2)));
    FCA_TRY(dev_alloc(c, &c->P, (size_t)c->nprob * kMaxM * kMaxM * sizeof(double2)));
    FCA_TRY(dev_alloc(c, &c->Pinv, (size_t)c->nprob * kMaxM * kMaxM * sizeof(double2)));
    FCA_TRY(dev_alloc(c, &c->P0, (size_t)c->nprob * kMaxM * kMaxM * sizeof(double2)));
    FCA_TRY(dev_alloc(c, &c->lam0, (size_t)c->nprob * kMaxM * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->logdet0, (size_t)c->nprob * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->lam, (size_t)c->nprob * kMaxM * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->logdet, (size_t)c->nprob * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->flags, (size_t)c->nprob * sizeof(int)));
    FCA_TRY(dev_alloc(c, &c->ll, (size_t)kLChunk * c->nprob * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->ll_tot, (size_t)kLChunk * B * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->fsum, (size_t)B * (c->F + 1) * sizeof(double)));
    FCA_TRY(dev_alloc(c, &c->R_stage, 2ull * c->F * maxM * maxM * sizeof(double2)));
    FCA_TRY(dev_alloc(c, &c->probs, (size_t)c->nprob * sizeof(EmProblem)));
    FCA_TRY(dev_alloc(c, &c->probs_act, (size_t)c->nprob * sizeof(EmProblem)));
    FCA_TRY(dev_alloc(c, &c->x_off, (size_t)c->nprob * 2 * sizeof(int64_t)));
    FCA_TRY(dev_alloc(c, &c->flag_sum, 5 * sizeof(int)));
    FCA_TRY(dev_alloc(c, &c->inactive_dev, (size_t)B * sizeof(int)));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->ll_host), (size_t)kLChunk * B * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->ll_host = nullptr;
        set_err(c, "hipHostMalloc failed");
        FCA_TRY(FCA_E_NOMEM);
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->flag_sum_host), 5 * sizeof(int), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        c->flag_sum_host = nullptr;
        set_err(c, "hipHostMalloc failed");
        FCA_TRY(FCA_E_NOMEM);
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->table_act), (size_t)c->nprob * sizeof(EmProblem),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->table_act = nullptr;
        set_err(c, "hipHostMalloc failed");
        FCA_TRY(FCA_E_NOMEM);
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->inactive_host), (size_t)B * sizeof(int), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        c->inactive_host = nullptr;
        set_err(c, "hipHostMalloc failed");
        FCA_TRY(FCA_E_NOMEM);
    }
    if (hipEventCreateWithFlags(&c->table_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        c->table_ev = nullptr;
        set_err(c, "hipEventCreate failed");
        FCA_TRY(FCA_E_DEVICE);
    }
    auto hipcall = [&](hipError_t e, const char* what) -> fca_status {
        if (e == hipSuccess) return FCA_OK;
        set_err(c, "%s failed: %s", what, hipGetErrorString(e));
        return FCA_E_DEVICE;
    };
    FCA_TRY(hipcall(hipEventCreate(&c->ev0), "hipEventCreate"));
    FCA_TRY(hipcall(hipEventCreate(&c->ev1), "hipEventCreate"));

    const hipStream_t s = c->stream;
    // ---- problem table: groups of equal (M, fpt), larger N first inside a group
    std::vector<EmProblem> table;
    std::vector<int64_t> xoff;
    {
        std::vector<int> order(B);
        for (int b = 0; b < B; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const MixInfo &A = c->mix[a], &Bm = c->mix[b];
            if (A.M != Bm.M) return A.M < Bm.M;
            if (A.fpt != Bm.fpt) return A.fpt > Bm.fpt;
            return A.N > Bm.N;
        });
        for (int oi = 0; oi < B; ++oi) {
            const int b = order[oi];
            const MixInfo& mi = c->mix[b];
            if (c->groups.empty() || c->groups.back().M != mi.M || c->groups.back().fpt != mi.fpt)
                c->groups.push_back(Group{mi.M, mi.fpt, (int)table.size(), 0, 0, kEmThreads, mi.fpt});
            Group& g = c->groups.back();
            for (int f = 0; f < c->F; ++f) {
                EmProblem e;
                e.y_off = mi.y_base + (int64_t)f * mi.M * mi.npad;
                e.v_off = mi.v_base + (int64_t)f * mi.npad;
                e.v2_off = (int64_t)c->F * mi.npad;
                e.n = mi.N;
                e.npad = mi.npad;
                e.pid = mi.pid0 + f;
                e.m = mi.M;
                table.push_back(e);
                xoff.push_back(mi.out_x + (int64_t)f * mi.N * mi.M);
                xoff.push_back(mi.out_x + ((int64_t)c->F + f) * mi.N * mi.M);
            }
            g.count += c->F;
            g.max_n = std::max(g.max_n, mi.N);
        }
    }
    // Default launch shape: 256 threads with the group's frames per thread.
    // A float-bulk group at M <= 4 with more problems than 256-thread
    // workgroups hold at once (three per CU) and at most 1024 frames starts at
    // 128 threads (eight frames per thread) instead: those workgroups hold
    // more problems per CU in registers (at M = 4 four rather than three;
    // measured 7 % faster per iteration on 256 mixtures of 513 x 1000 bins).
    // fca_set_launch_shape and fca_autotune override it.
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            cus = 0;
        }
        for (Group& g : c->groups) {
            if (c->fp64 || g.M > 4 || g.fpt == 0 || g.max_n > 128 * kMaxFramesPerThread || cus <= 0 ||
                g.count <= 3 * cus)
                continue;
            int f = 1;
            while (f * 128 < g.max_n) f *= 2;
            g.nt = 128;
            g.run_fpt = f;
        }
    }
    c->table = table;
    FCA_TRY(hipcall(hipMemcpyAsync(c->probs, c->table.data(), c->table.size() * sizeof(EmProblem),
                                   hipMemcpyHostToDevice, s), "hipMemcpyAsync(problems)"));
    FCA_TRY(hipcall(hipMemcpyAsync(c->x_off, xoff.data(), xoff.size() * sizeof(int64_t),
                                   hipMemcpyHostToDevice, s), "hipMemcpyAsync(x offsets)"));

    // ---- copy y (K0 ingest), R0, v0
    for (int b = 0; b < B; ++b) {
        const fca_problem& p = probs[b];
        const MixInfo& mi = c->mix[b];
        const int64_t extent = (int64_t)(p.F - 1) * p.y_stride_f + (int64_t)(p.N - 1) * p.y_stride_n +
                               (int64_t)(p.M - 1) * p.y_stride_m + 1;
        const void* src = p.y;
        void* tmp = nullptr;
        if (!is_device_ptr(p.y)) {
            FCA_TRY(dev_alloc(c, &tmp, extent * c->esz));
            fca_status cs = hipcall(hipMemcpyAsync(tmp, p.y, extent * c->esz, hipMemcpyHostToDevice, s),
                                    "hipMemcpyAsync(y)");
            if (cs != FCA_OK) { (void)hipFree(tmp); FCA_TRY(cs); }
            src = tmp;
        }
        fca_status ks = hipcall(launch_ingest(c->fp64, src, p.y_stride_f, p.y_stride_n, p.y_stride_m, mi.M,
                                              c->F, mi.N, mi.npad,
                                              static_cast<char*>(c->y) + mi.y_base * c->esz, s),
                                "ingest");
        if (tmp) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(tmp);
        }
        FCA_TRY(ks);

        double2* Rb = c->R_init + mi.R_base;
        c->mix[b].R_default = p.R0 == nullptr;
        if (p.R0) {
            FCA_TRY(hipcall(hipMemcpyAsync(Rb, p.R0, 2ull * c->F * mi.M * mi.M * sizeof(double2),
                                           hipMemcpyDefault, s), "hipMemcpyAsync(R0)"));
        } else {
            FCA_TRY(hipcall(launch_default_R(mi.M, c->F, Rb, s), "default R0"));
        }
        if (p.v0) {
            const size_t vbytes = 2ull * c->F * mi.N * c->rsz;
            const void* vsrc = p.v0;
            void* vtmp = nullptr;
            if (!is_device_ptr(p.v0)) {
                FCA_TRY(dev_alloc(c, &vtmp, vbytes));
                fca_status cs = hipcall(hipMemcpyAsync(vtmp, p.v0, vbytes, hipMemcpyHostToDevice, s),
                                        "hipMemcpyAsync(v0)");
                if (cs != FCA_OK) { (void)hipFree(vtmp); FCA_TRY(cs); }
                vsrc = vtmp;
            }
            fca_status ks2 = hipcall(launch_copy_v_in(c->fp64, vsrc, c->F, mi.N, mi.npad,
                                                      static_cast<char*>(c->v_init) + mi.v_base * c->rsz, s),
                                     "copy v0");
            if (vtmp) {
                (void)hipStreamSynchronize(s);
                (void)hipFree(vtmp);
            }
            FCA_TRY(ks2);
        }
    }
    FCA_TRY(hipcall(hipStreamSynchronize(s), "hipStreamSynchronize"));

    for (int b = 0; b < B; ++b) FCA_TRY(compute_start(c, b, nullptr, s));
    st = check_initial_flags(c, 0, B);
    if (st == FCA_E_NOT_PD) st = FCA_E_ARG;
    FCA_TRY(st);
    FCA_TRY(do_reset(c));
#undef FCA_TRY
    *out = c;
    return FCA_OK;
}

}  // namespace

extern "C" {

fca_status fca_init(const fca_problem* p, fca_ctx** out) {
    if (!out) { set_err(nullptr, "out is NULL"); return FCA_E_ARG; }
    *out = nullptr;
    if (!p) { set_err(nullptr, "problem is NULL"); return FCA_E_ARG; }
    return init_impl(p, 1, out);
}

fca_status fca_init_batch(const fca_problem* p, int32_t B, fca_ctx** out) {
    if (!out) { set_err(nullptr, "out is NULL"); return FCA_E_ARG; }
    *out = nullptr;
    if (!p || B < 1) { set_err(nullptr, "need B >= 1 problems"); return FCA_E_ARG; }
    return init_impl(p, B, out);
}

fca_status fca_reset(fca_ctx* c) {
    if (!c) return FCA_E_ARG;
    if (c->broken) return FCA_E_STATE;
    return do_reset(c);
}

fca_status fca_set_start(fca_ctx* c, int32_t b, const double* R0, const void* v0) {
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (b < 0 || b >= c->B) { set_err(c, "fca_set_start: mixture %d outside 0..%d", b, c->B - 1); return FCA_E_ARG; }
    const hipStream_t s = c->stream;
    MixInfo& mi = c->mix[b];
    const int64_t mm = (int64_t)mi.M * mi.M;
    const size_t rbytes = 2ull * c->F * mm * sizeof(double2);
    double2* Rb = c->R_init + mi.R_base;
    if (R0) {
        // stage, decompose and check before the mixture's stored start changes
        FCA_HIP(c, hipMemcpyAsync(c->R_stage, R0, rbytes, hipMemcpyDefault, s));
        fca_status st = compute_basis(c, b, c->R_stage, s);
        if (st != FCA_OK) return st;
        st = check_initial_flags(c, b, b + 1);
        if (st == FCA_E_NOT_PD) {
            st = compute_basis(c, b, nullptr, s);  // the stored basis of the old R0 again
            if (st == FCA_OK) st = check_initial_flags(c, b, b + 1);
            if (st == FCA_OK) {
                set_err(c, "fca_set_start: R0 of mixture %d is not positive definite", b);
                st = FCA_E_ARG;
            }
            return st;
        }
        if (st != FCA_OK) return st;
        FCA_HIP(c, hipMemcpyAsync(Rb, c->R_stage, rbytes, hipMemcpyDeviceToDevice, s));
        mi.R_default = false;
    } else if (!mi.R_default) {
        FCA_HIP(c, launch_default_R(mi.M, c->F, Rb, s));
        mi.R_default = true;
    }
    if (v0) {
        fca_status st0 = ensure_v_init(c);
        if (st0 != FCA_OK) return st0;
        const size_t vbytes = 2ull * c->F * mi.N * c->rsz;
        const void* vsrc = v0;
        void* vtmp = nullptr;
        if (!is_device_ptr(v0)) {
            fca_status st = dev_alloc(c, &vtmp, vbytes);
            if (st != FCA_OK) return st;
            hipError_t e = hipMemcpyAsync(vtmp, v0, vbytes, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                (void)hipFree(vtmp);
                FCA_HIP(c, e);
            }
            vsrc = vtmp;
        }
        hipError_t e = launch_copy_v_in(c->fp64, vsrc, c->F, mi.N, mi.npad,
                                        static_cast<char*>(c->v_init) + mi.v_base * c->rsz, s);
        if (vtmp) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(vtmp);
        }
        FCA_HIP(c, e);
    }
    mi.has_v0 = v0 != nullptr;
    c->shape_version += 1;  // the start changed since any capture
    fca_status st = compute_start(c, b, nullptr, s);
    if (st == FCA_OK) st = restore_start(c, b, s);
    if (st != FCA_OK) return st;
    if (!c->active[b]) {
        c->active[b] = 1;
        c->act_dirty = true;
    }
    return FCA_OK;
}

fca_status fca_set_learned_starts(fca_ctx* c, fca_mlp* m, int32_t count, const int32_t* mixtures) {
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (!m) { set_err(c, "fca_set_learned_starts: no network"); return FCA_E_ARG; }
    if (c->fp64) { set_err(c, "fca_set_learned_starts: needs an FP32-bulk context"); return FCA_E_ARG; }
    if (count < 1 || count > c->B) {
        set_err(c, "fca_set_learned_starts: count %d outside 1..%d", count, c->B);
        return FCA_E_ARG;
    }
    std::vector<int> list(count);
    for (int i = 0; i < count; ++i) {
        const int b = mixtures ? mixtures[i] : i;
        if (b < 0 || b >= c->B) {
            set_err(c, "fca_set_learned_starts: mixture %d outside 0..%d", b, c->B - 1);
            return FCA_E_ARG;
        }
        if (c->mix[b].M != mlp_microphones(m)) {
            set_err(c, "fca_set_learned_starts: mixture %d has M = %d, the network M = %d", b, c->mix[b].M,
                    mlp_microphones(m));
            return FCA_E_ARG;
        }
        list[i] = b;
    }
    const hipStream_t s = c->stream;
    {
        fca_status st = ensure_v_init(c);
        if (st != FCA_OK) return st;
    }
    // one inference launch writes v_init and v of every listed mixture
    std::vector<MlpInferJob> jobs(count);
    for (int i = 0; i < count; ++i) {
        const MixInfo& mi = c->mix[list[i]];
        const int64_t np = mi.npad;
        jobs[i] = MlpInferJob{reinterpret_cast<const float2*>(c->y) + mi.y_base,
                              static_cast<float*>(c->v_init) + mi.v_base,
                              static_cast<float*>(c->v) + mi.v_base,
                              (int64_t)mi.M * np, 1, np, (int64_t)c->F * np, np, 0, c->F, mi.N};
    }
    const char* err = nullptr;
    const hipError_t e = mlp_infer_jobs(m, jobs.data(), count, s, &err);
    if (err) {
        set_err(c, "fca_set_learned_starts: %s", err);
        return e == hipErrorOutOfMemory ? FCA_E_NOMEM : FCA_E_ARG;
    }
    FCA_HIP(c, e);
    // the rest of theta^(0): the basis of the plain R (stored already unless
    // a caller's R0 was in place), copied into the working state
    for (int b : list) {
        MixInfo& mi = c->mix[b];
        if (!mi.R_default) {
            FCA_HIP(c, launch_default_R(mi.M, c->F, c->R_init + mi.R_base, s));
            mi.R_default = true;
            fca_status st = compute_basis(c, b, nullptr, s);
            if (st != FCA_OK) return st;
        }
        mi.has_v0 = true;
        if (!c->active[b]) {
            c->active[b] = 1;
            c->act_dirty = true;
        }
    }
    if (!mixtures && count == c->B) {
        fca_status st = restore_all(c, s);
        if (st != FCA_OK) return st;
    } else {
        for (int b : list) {
            fca_status st = restore_start(c, b, s);
            if (st != FCA_OK) return st;
        }
    }
    c->shape_version += 1;  // the starts changed since any capture
    return FCA_OK;
}

fca_status fca_set_mask_covariances(fca_ctx* c, int32_t count, const int32_t* mixtures, double sharpen, double load) {
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (count < 1 || count > c->B) {
        set_err(c, "fca_set_mask_covariances: count %d outside 1..%d", count, c->B);
        return FCA_E_ARG;
    }
    if (!(sharpen >= 1.0 && sharpen <= 64.0)) {
        set_err(c, "fca_set_mask_covariances: sharpen %g outside [1, 64]", sharpen);
        return FCA_E_ARG;
    }
    if (!(load > 0.0 && load <= 1e6)) {
        set_err(c, "fca_set_mask_covariances: load %g outside (0, 1e6]", load);
        return FCA_E_ARG;
    }
    std::vector<int> list(count);
    for (int i = 0; i < count; ++i) {
        const int b = mixtures ? mixtures[i] : i;
        if (b < 0 || b >= c->B) {
            set_err(c, "fca_set_mask_covariances: mixture %d outside 0..%d", b, c->B - 1);
            return FCA_E_ARG;
        }
        if (!c->mix[b].has_v0) {
            // equal powers give the masks 1/2 everywhere and R1 = R2: a fixed
            // point of the EM that never separates the sources
            set_err(c, "fca_set_mask_covariances: mixture %d has the plain start's equal powers; give it distinct "
                       "powers first (v0, fca_set_start or fca_set_learned_starts)", b);
            return FCA_E_ARG;
        }
        list[i] = b;
    }
    const hipStream_t s = c->stream;
    {
        fca_status st = ensure_v_init(c);
        if (st != FCA_OK) return st;
    }
    if (!c->mask_mix) {
        fca_status st = dev_alloc(c, &c->mask_mix, sizeof(MaskCovMix) * c->B);
        if (st != FCA_OK) return st;
        if (hipHostMalloc(reinterpret_cast<void**>(&c->mask_mix_host), sizeof(MaskCovMix) * c->B) != hipSuccess) {
            (void)hipGetLastError();
            c->mask_mix_host = nullptr;
            (void)hipFree(c->mask_mix);
            c->mask_mix = nullptr;
            set_err(c, "fca_set_mask_covariances: pinned allocation failed");
            return FCA_E_NOMEM;
        }
    }
    // one launch per microphone count; the staging is free again when this
    // call returns (it ends with the stream synchronised)
    // one microphone: A_j is a positive scalar or zero, so R_j = 1 + load
    // for both sources (no kernel needed)
    for (int b : list) {
        const MixInfo& mi = c->mix[b];
        if (mi.M != 1) continue;
        const std::vector<double2> one(2 * (size_t)c->F, make_double2(1.0 + load, 0.0));
        FCA_HIP(c, hipMemcpyAsync(c->R_init + mi.R_base, one.data(), sizeof(double2) * one.size(),
                                  hipMemcpyHostToDevice, s));
        FCA_HIP(c, hipStreamSynchronize(s));
    }
    int k = 0;
    for (int M = 2; M <= kMaxM; ++M) {
        const int k0 = k;
        for (int b : list) {
            const MixInfo& mi = c->mix[b];
            if (mi.M == M) c->mask_mix_host[k++] = MaskCovMix{mi.y_base, mi.v_base, mi.R_base, mi.N, mi.npad};
        }
        if (k == k0) continue;
        FCA_HIP(c, hipMemcpyAsync(c->mask_mix + k0, c->mask_mix_host + k0, sizeof(MaskCovMix) * (k - k0),
                                  hipMemcpyHostToDevice, s));
        FCA_HIP(c, launch_mask_cov(c->fp64, M, c->mask_mix + k0, k - k0, c->F, c->y, c->v_init, c->R_init, sharpen,
                                   load, s));
    }
    // the bases: one decomposition launch per run of consecutive listed
    // mixtures of equal M (their R blocks lie 2 F M^2 apart, their problems
    // consecutive)
    for (size_t i = 0; i < list.size();) {
        const int b0 = list[i];
        const MixInfo& m0 = c->mix[b0];
        size_t e = i + 1;
        while (e < list.size() && list[e] == list[e - 1] + 1 && c->mix[list[e]].M == m0.M) ++e;
        const int nb = (int)(e - i);
        const int64_t mm = (int64_t)m0.M * m0.M;
        const double2* R1 = c->R_init + m0.R_base;
        FCA_HIP(c, launch_gevd_runs(m0.M, nb * c->F, c->F, 2LL * c->F * mm, R1, R1 + (int64_t)c->F * mm, mm, mm,
                                    c->P0 + (int64_t)m0.pid0 * kMaxM * kMaxM, kMaxM * kMaxM,
                                    c->lam0 + (int64_t)m0.pid0 * kMaxM, kMaxM, c->logdet0 + m0.pid0,
                                    c->flags + m0.pid0, s));
        for (size_t k = i; k < e; ++k) c->mix[list[k]].R_default = false;
        i = e;
    }
    const bool all = !mixtures && count == c->B;
    fca_status st = FCA_OK;
    if (all) {
        st = check_initial_flags(c, 0, c->B);
    } else {
        for (int b : list)
            if ((st = check_initial_flags(c, b, b + 1)) != FCA_OK) break;
    }
    if (st == FCA_E_NOT_PD) {
        // back to the default R for every listed mixture
        const std::string why = c->err;
        for (int b : list) {
            MixInfo& mi = c->mix[b];
            FCA_HIP(c, launch_default_R(mi.M, c->F, c->R_init + mi.R_base, s));
            mi.R_default = true;
            fca_status st2 = compute_basis(c, b, nullptr, s);
            if (st2 == FCA_OK) st2 = check_initial_flags(c, b, b + 1);
            if (st2 != FCA_OK) return st2;
        }
        set_err(c, "fca_set_mask_covariances: %s; the listed mixtures keep the default R", why.c_str());
    } else if (st != FCA_OK) {
        return st;
    }
    for (int b : list) {
        if (!c->active[b]) {
            c->active[b] = 1;
            c->act_dirty = true;
        }
    }
    fca_status st3 = FCA_OK;
    if (all) {
        st3 = restore_all(c, s);
    } else {
        for (int b : list)
            if ((st3 = restore_start(c, b, s)) != FCA_OK) break;
    }
    if (st3 != FCA_OK) return st3;
    c->shape_version += 1;  // the starts changed since any capture
    return st == FCA_E_NOT_PD ? FCA_E_NOT_PD : FCA_OK;
}

fca_status fca_set_active(fca_ctx* c, int32_t b, int32_t active) {
    if (!c) return FCA_E_ARG;
    if (b < 0 || b >= c->B) { set_err(c, "fca_set_active: mixture %d outside 0..%d", b, c->B - 1); return FCA_E_ARG; }
    const char a = active != 0;
    if (c->active[b] != a) {
        c->active[b] = a;
        c->act_dirty = true;
    }
    return FCA_OK;
}

}  // extern "C"

namespace fca {

hipError_t launch_em(int M, bool fp64, int nt, int fpt, const EmProblem* probs, int count, const void* y,
                     void* v, int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                     int64_t ll_stride, int iters, int it_base, hipStream_t s) {
    if (nt == kEmThreads)
        return launch_em_nt<kEmThreads>(M, fp64, fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll,
                                        ll_stride, iters, it_base, s);
    if (nt == 128)
        return launch_em_nt<128>(M, fp64, fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll, ll_stride,
                                 iters, it_base, s);
    return hipErrorInvalidValue;
}

hipError_t launch_conv_em(int M, bool fp64, int fpt, const EmProblem* probs, int count, const void* y, void* v,
                          int64_t v_alt, double2* P, double* lam, double* logdet, int* flags, double* ll,
                          int64_t ll_stride, int iters, int it_base, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (M) {
#define FCA_CONV_CASE(MM_)                                                                                         \
    case MM_:                                                                                                      \
        return fp64 ? launch_conv_fpt<MM_, double>(fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll,     \
                                                    ll_stride, iters, it_base, s)                                  \
                    : launch_conv_fpt<MM_, float>(fpt, probs, count, y, v, v_alt, P, lam, logdet, flags, ll,       \
                                                   ll_stride, iters, it_base, s);
        FCA_CONV_CASE(1) FCA_CONV_CASE(2) FCA_CONV_CASE(3) FCA_CONV_CASE(4)
        FCA_CONV_CASE(5) FCA_CONV_CASE(6) FCA_CONV_CASE(7) FCA_CONV_CASE(8)
#undef FCA_CONV_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fca

namespace {

// Side streams and events for concurrent launch groups (created once).
fca_status ensure_side_streams(fca_ctx* c, int want) {
    want = std::min(want, kMaxSide);
    if (!c->fork_ev) FCA_HIP(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    while (c->nside < want) {
        const int i = c->nside;
        FCA_HIP(c, hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
        FCA_HIP(c, hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming));
        c->nside += 1;
    }
    return FCA_OK;
}

// One chunk of `chunk` iterations for every problem of `groups`: the largest
// group on stream s, the others spread over the side streams, all forked from
// and joined back to s (so the groups' tails overlap instead of serialising).
fca_status enqueue_em_groups(fca_ctx* c, const std::vector<Group>& groups, const EmProblem* probs, int chunk,
                             int it_base, bool conventional, hipStream_t s) {
    const int ng = (int)groups.size();
    int nside = 0;
    if (ng > 1 && !conventional) {
        fca_status st = ensure_side_streams(c, ng - 1);
        if (st != FCA_OK) return st;
        nside = std::min(ng - 1, c->nside);
        FCA_HIP(c, hipEventRecord(c->fork_ev, s));
        for (int i = 0; i < nside; ++i) FCA_HIP(c, hipStreamWaitEvent(c->side[i], c->fork_ev, 0));
    }
    // largest group first on the main stream
    int big = 0;
    for (int i = 1; i < ng; ++i)
        if ((int64_t)groups[i].count * groups[i].max_n > (int64_t)groups[big].count * groups[big].max_n) big = i;
    int k = 0;
    for (int i = 0; i < ng; ++i) {
        const Group& g = groups[i];
        hipStream_t gs = s;
        if (nside > 0 && i != big) gs = c->side[(k++) % nside];
        if (conventional)
            FCA_HIP(c, launch_conv_em(g.M, c->fp64, g.fpt, probs + g.first, g.count, c->y, c->v, c->v_alt, c->P,
                                      c->lam, c->logdet, c->flags, c->ll, c->nprob, chunk, it_base, gs));
        else
            FCA_HIP(c, launch_em(g.M, c->fp64, g.nt, g.run_fpt, probs + g.first, g.count, c->y, c->v, c->v_alt,
                                 c->P, c->lam, c->logdet, c->flags, c->ll, c->nprob, chunk, it_base, gs));
    }
    for (int i = 0; i < nside; ++i) {
        FCA_HIP(c, hipEventRecord(c->join_ev[i], c->side[i]));
        FCA_HIP(c, hipStreamWaitEvent(s, c->join_ev[i], 0));
    }
    return FCA_OK;
}

// Log-likelihood totals of one chunk into a device [B][total] array at
// column `done` (inactive mixtures: NaN rows).
fca_status enqueue_ll_out(fca_ctx* c, int rows, int total, int done, double* loglik_dev, hipStream_t s) {
    FCA_HIP(c, launch_ll_reduce(c->ll, c->nprob, rows, c->B, c->F, c->ll_tot, s));
    if (!c->all_active && c->n_inactive)  // NaN in every row of an inactive mixture, one launch
        FCA_HIP(c, launch_nan_rows(c->ll_tot, 0, 1, rows, rows, c->inactive_dev, c->n_inactive, s));
    if (loglik_dev)
        FCA_HIP(c, hipMemcpy2DAsync(loglik_dev + done, total * sizeof(double), c->ll_tot, rows * sizeof(double),
                                    rows * sizeof(double), c->B, hipMemcpyDeviceToDevice, s));
    return FCA_OK;
}

// R_j(f) of every mixture into a device batch array (eq. recoverS); with
// keep_pinv the inverses P^-1 are stored for a following separation.
fca_status enqueue_R_out(fca_ctx* c, double2* R_dev, hipStream_t s, bool keep_pinv = false) {
    for (int b = 0; b < c->B; ++b) {
        const MixInfo& mi = c->mix[b];
        const int64_t mm = (int64_t)mi.M * mi.M;
        double2* dst = R_dev + mi.out_R;
        FCA_HIP(c, launch_pinv(mi.M, c->F, c->P + (int64_t)mi.pid0 * kMaxM * kMaxM, c->lam + (int64_t)mi.pid0 * kMaxM,
                               keep_pinv ? c->Pinv + (int64_t)mi.pid0 * kMaxM * kMaxM : nullptr, dst,
                               dst + (int64_t)c->F * mm, s));
    }
    return FCA_OK;
}

fca_status enqueue_v_out(fca_ctx* c, void* v_out, hipStream_t s) {
    for (int b = 0; b < c->B; ++b) {
        const MixInfo& mi = c->mix[b];
        FCA_HIP(c, hipMemcpy2DAsync(static_cast<char*>(v_out) + mi.out_v * c->rsz, mi.N * c->rsz,
                                    static_cast<char*>(c->v) + mi.v_base * c->rsz, mi.npad * c->rsz,
                                    mi.N * c->rsz, 2 * c->F, hipMemcpyDefault, s));
    }
    return FCA_OK;
}

fca_status enqueue_separate(fca_ctx* c, void* x_dev, hipStream_t s, bool have_pinv = false) {
    for (const MixInfo& mi : c->mix)
        if (!have_pinv)
            FCA_HIP(c, launch_pinv(mi.M, c->F, c->P + (int64_t)mi.pid0 * kMaxM * kMaxM, c->lam + (int64_t)mi.pid0 * kMaxM,
                               c->Pinv + (int64_t)mi.pid0 * kMaxM * kMaxM, nullptr, nullptr, s));
    for (const Group& g : c->groups)
        FCA_HIP(c, launch_separate(g.M, c->fp64, c->probs + g.first, g.count, g.max_n, c->y, c->v, c->P, c->lam,
                                   c->Pinv, x_dev, c->x_off + 2 * (int64_t)g.first, s));
    return FCA_OK;
}

// Shared driver of fca_em_step (FastFCA kernels) and fca_conv_em_step
// (conventional frame-wise EM kernel): chunks of at most kLChunk iterations,
// log-likelihood totals per mixture, then R and v out.
fca_status em_step_impl(fca_ctx* c, int32_t iters, double* loglik, double* R_out, void* v_out, bool conventional) {
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (iters < 0) { set_err(c, "iters < 0"); return FCA_E_ARG; }
    {
        fca_status st = refresh_active(c);
        if (st != FCA_OK) return st;
    }
    const std::vector<Group>& groups = c->all_active ? c->groups : c->groups_act;
    const EmProblem* probs = c->all_active ? c->probs : c->probs_act;
    const hipStream_t s = c->stream;
    const bool ll_dev = loglik && is_device_ptr(loglik);
    int done = 0;
    do {
        const int chunk = iters == 0 ? 0 : std::min(kLChunk, iters - done);
        const int rows = chunk > 0 ? chunk : 1;
        if (c->timing) FCA_HIP(c, hipEventRecord(c->ev0, s));
        {
            fca_status st = enqueue_em_groups(c, groups, probs, chunk, done, conventional, s);
            if (st != FCA_OK) return st;
        }
        if (c->timing) FCA_HIP(c, hipEventRecord(c->ev1, s));
        if (loglik) {
            const int total = iters > 0 ? iters : 1;
            fca_status st = enqueue_ll_out(c, rows, total, done, ll_dev ? loglik : nullptr, s);
            if (st != FCA_OK) return st;
            if (!ll_dev) {
                FCA_HIP(c, hipMemcpyAsync(c->ll_host, c->ll_tot, (size_t)rows * c->B * sizeof(double),
                                          hipMemcpyDeviceToHost, s));
                FCA_HIP(c, hipStreamSynchronize(s));
                for (int b = 0; b < c->B; ++b)
                    memcpy(loglik + (size_t)b * total + done, c->ll_host + (size_t)b * rows, rows * sizeof(double));
            }
        }
        if (c->timing) {
            FCA_HIP(c, hipEventSynchronize(c->ev1));
            float ms = 0.f;
            FCA_HIP(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
            c->em_ms += ms;
            c->em_launches += (int64_t)groups.size();
        }
        c->last_rows = rows;
        done += chunk;
    } while (done < iters);
    c->last_active = c->active;

    if (R_out) {
        const bool dev = is_device_ptr(R_out);
        for (int b = 0; b < c->B; ++b) {
            const MixInfo& mi = c->mix[b];
            const int64_t mm = (int64_t)mi.M * mi.M;
            double2* dst = dev ? reinterpret_cast<double2*>(R_out) + mi.out_R : c->R_stage;
            FCA_HIP(c, launch_recover_R(mi.M, c->F, c->P + (int64_t)mi.pid0 * kMaxM * kMaxM,
                                        c->lam + (int64_t)mi.pid0 * kMaxM, dst, dst + (int64_t)c->F * mm, s));
            if (!dev) {
                FCA_HIP(c, hipMemcpyAsync(reinterpret_cast<double2*>(R_out) + mi.out_R, c->R_stage,
                                          2ull * c->F * mm * sizeof(double2), hipMemcpyDeviceToHost, s));
                FCA_HIP(c, hipStreamSynchronize(s));
            }
        }
    }
    if (v_out) {
        for (int b = 0; b < c->B; ++b) {
            const MixInfo& mi = c->mix[b];
            FCA_HIP(c, hipMemcpy2DAsync(static_cast<char*>(v_out) + mi.out_v * c->rsz, mi.N * c->rsz,
                                        static_cast<char*>(c->v) + mi.v_base * c->rsz, mi.npad * c->rsz,
                                        mi.N * c->rsz, 2 * c->F, hipMemcpyDefault, s));
        }
    }
    return check_flags(c);
}

}  // namespace

extern "C" {

fca_status fca_em_step(fca_ctx* c, int32_t iters, double* loglik, double* R_out, void* v_out) {
    return em_step_impl(c, iters, loglik, R_out, v_out, false);
}

fca_status fca_conv_em_step(fca_ctx* c, int32_t iters, double* loglik, double* R_out, void* v_out) {
    return em_step_impl(c, iters, loglik, R_out, v_out, true);
}

fca_status fca_separate(fca_ctx* c, void* x_out) {
    if (!c || !x_out) { if (c) set_err(c, "x_out is NULL"); return FCA_E_ARG; }
    if (c->broken) return FCA_E_STATE;
    const hipStream_t s = c->stream;
    int64_t total = 0;
    for (const MixInfo& mi : c->mix) total += 2LL * c->F * mi.N * mi.M;
    const bool dev = is_device_ptr(x_out);
    void* dst = x_out;
    if (!dev) {
        fca_status st = dev_alloc(c, &dst, total * c->esz);
        if (st != FCA_OK) return st;
    }
    hipError_t e = hipSuccess;
    for (const MixInfo& mi : c->mix) {
        e = launch_pinv(mi.M, c->F, c->P + (int64_t)mi.pid0 * kMaxM * kMaxM, c->lam + (int64_t)mi.pid0 * kMaxM,
                        c->Pinv + (int64_t)mi.pid0 * kMaxM * kMaxM, nullptr, nullptr, s);
        if (e != hipSuccess) break;
    }
    for (const Group& g : c->groups) {
        if (e != hipSuccess) break;
        e = launch_separate(g.M, c->fp64, c->probs + g.first, g.count, g.max_n, c->y, c->v, c->P, c->lam, c->Pinv,
                            dst, c->x_off + 2 * (int64_t)g.first, s);
    }
    if (e == hipSuccess && !dev) e = hipMemcpyAsync(x_out, dst, total * c->esz, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (!dev) (void)hipFree(dst);
    if (e != hipSuccess) {
        set_err(c, "fca_separate: %s", hipGetErrorString(e));
        c->broken = true;
        return FCA_E_DEVICE;
    }
    return FCA_OK;
}

fca_status fca_status_per_freq(const fca_ctx* c, int32_t* flags) {
    if (!c || !flags) return FCA_E_ARG;
    fca_ctx* cc = const_cast<fca_ctx*>(c);
    if (cc->broken) return FCA_E_STATE;
    FCA_HIP(cc, hipMemcpyAsync(cc->flags_host.data(), cc->flags, sizeof(int) * cc->nprob,
                               hipMemcpyDeviceToHost, cc->stream));
    FCA_HIP(cc, hipStreamSynchronize(cc->stream));
    for (int i = 0; i < cc->nprob; ++i) flags[i] = cc->flags_host[i] & kFlagBitsMask;
    return FCA_OK;
}

const char* fca_last_error(const fca_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"

void fca::set_global_error(const char* msg) { g_init_error = msg; }

extern "C" {

void fca_destroy(fca_ctx* c) {
    if (!c) return;
    if (c->stream || true) (void)hipStreamSynchronize(c->stream);
    free_ctx_memory(c);
    delete c;
}

fca_status fca_gevd(int32_t M, int32_t count, const double* S1, const double* S2, double* P, double* lambda,
                    int32_t* flags, void* stream) {
    if (M < 1 || M > kMaxM || count < 0) { set_err(nullptr, "fca_gevd: bad M or count"); return FCA_E_ARG; }
    if (count == 0) return FCA_OK;
    if (!is_device_ptr(S1) || !is_device_ptr(S2) || !is_device_ptr(P) || !is_device_ptr(lambda) ||
        !is_device_ptr(flags)) {
        set_err(nullptr, "fca_gevd: all arrays must be device pointers");
        return FCA_E_ARG;
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t mm = (int64_t)M * M;
    hipError_t e = launch_gevd(M, count, reinterpret_cast<const double2*>(S1), reinterpret_cast<const double2*>(S2),
                               mm, mm, reinterpret_cast<double2*>(P), mm, lambda, M, nullptr, flags, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_err(nullptr, "fca_gevd: %s", hipGetErrorString(e));
        return FCA_E_DEVICE;
    }
    return FCA_OK;
}

fca_status fca_timing(fca_ctx* c, int32_t enable, double* em_kernel_ms, int64_t* em_launches) {
    if (!c) return FCA_E_ARG;
    if (em_kernel_ms) *em_kernel_ms = c->em_ms;
    if (em_launches) *em_launches = c->em_launches;
    c->em_ms = 0.0;
    c->em_launches = 0;
    c->timing = enable != 0;
    return FCA_OK;
}


// ---------------------------------------------------------------- launch shapes and autotuning
fca_status fca_launch_groups(const fca_ctx* c, fca_launch_group* out, int32_t cap, int32_t* count) {
    if (!c || (cap > 0 && !out)) return FCA_E_ARG;
    const int ng = (int)c->groups.size();
    if (count) *count = ng;
    for (int i = 0; i < ng && i < cap; ++i) {
        const Group& g = c->groups[i];
        out[i].M = g.M;
        out[i].threads = g.nt;
        out[i].frames_per_thread = g.fpt == 0 ? 0 : g.run_fpt;
        out[i].problems = g.count;
        out[i].max_frames = g.max_n;
    }
    return FCA_OK;
}

}  // extern "C"

namespace {

// Frames per thread for `nt` threads and up to max_n frames (0: streamed),
// or -1 when the shape cannot hold the group. Every group can stream with
// kEmThreads threads; groups beyond the resident limit can only stream.
int shape_fpt(const Group& g, int nt, bool streamed) {
    if (streamed) return nt == kEmThreads ? 0 : -1;
    if (g.fpt == 0) return -1;
    if (nt != kEmThreads && nt != 128) return -1;
    int f = 1;
    while (f * nt < g.max_n) f *= 2;
    return f <= kMaxFramesPerThread ? f : -1;
}

void shapes_changed(fca_ctx* c) {
    c->act_dirty = true;  // rebuilds the active-mixture tables with the new shapes
    c->shape_version += 1;
}

}  // namespace

extern "C" {

fca_status fca_set_launch_shape(fca_ctx* c, int32_t group, int32_t threads, int32_t streamed) {
    if (!c) return FCA_E_ARG;
    if (group < 0 || group >= (int)c->groups.size()) {
        set_err(c, "fca_set_launch_shape: group %d outside 0..%d", group, (int)c->groups.size() - 1);
        return FCA_E_ARG;
    }
    Group& g = c->groups[group];
    const int nt = threads == 0 ? kEmThreads : threads;
    const int f = shape_fpt(g, nt, streamed != 0);
    if (f < 0) {
        set_err(c, "fca_set_launch_shape: %d threads%s cannot hold group %d (%d frames%s)", threads,
                streamed ? " streaming" : "", group, g.max_n, g.fpt == 0 ? ", streamed only" : "");
        return FCA_E_ARG;
    }
    g.nt = nt;
    g.run_fpt = f;
    shapes_changed(c);
    return FCA_OK;
}

fca_status fca_autotune(fca_ctx* c, int32_t iters) {
    if (c) c->last_rows = 0;  // the trials overwrite the per-problem log-likelihood rows
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    iters = iters <= 0 ? 3 : std::min(iters, kLChunk);
    const hipStream_t s = c->stream;
    // the parameters are saved and put back after every trial run
    const size_t vb = (size_t)c->v_tot * c->rsz, pb = (size_t)c->nprob * kMaxM * kMaxM * sizeof(double2),
                 lb = (size_t)c->nprob * kMaxM * sizeof(double), db = (size_t)c->nprob * sizeof(double),
                 fb = (size_t)c->nprob * sizeof(int);
    char* save = nullptr;
    fca_status st = dev_alloc(c, &save, vb + pb + lb + db + fb);
    if (st != FCA_OK) return st;
    struct Buf { void* live; size_t off, bytes; };
    const Buf bufs[] = {{c->v, 0, vb}, {c->P, vb, pb}, {c->lam, vb + pb, lb}, {c->logdet, vb + pb + lb, db},
                        {c->flags, vb + pb + lb + db, fb}};
    auto copy_all = [&](bool to_save) -> hipError_t {
        for (const Buf& b : bufs) {
            hipError_t e = to_save ? hipMemcpyAsync(save + b.off, b.live, b.bytes, hipMemcpyDeviceToDevice, s)
                                   : hipMemcpyAsync(b.live, save + b.off, b.bytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = copy_all(true);
    for (size_t gi = 0; gi < c->groups.size() && e == hipSuccess; ++gi) {
        Group& g = c->groups[gi];
        int best_nt = g.nt, best_f = g.run_fpt;
        float best = -1.f;
        const int cand_nt[3] = {kEmThreads, 128, kEmThreads};
        const bool cand_stream[3] = {false, false, true};
        for (int ci = 0; ci < 3; ++ci) {
            const int nt = cand_nt[ci];
            const int f = shape_fpt(g, nt, cand_stream[ci]);
            if (f < 0) continue;
            float tmin = -1.f;
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // the first run loads the code object
                e = copy_all(false);
                if (e == hipSuccess) e = hipEventRecord(c->ev0, s);
                if (e == hipSuccess)
                    e = launch_em(g.M, c->fp64, nt, f, c->probs + g.first, g.count, c->y, c->v, c->v_alt, c->P,
                                  c->lam, c->logdet, c->flags, c->ll, c->nprob, iters, 0, s);
                if (e == hipSuccess) e = hipEventRecord(c->ev1, s);
                if (e == hipSuccess) e = hipEventSynchronize(c->ev1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
                if (e == hipSuccess && rep > 0 && (tmin < 0.f || ms < tmin)) tmin = ms;
            }
            if (e == hipSuccess && (best < 0.f || tmin < best)) {
                best = tmin;
                best_nt = nt;
                best_f = f;
            }
        }
        g.nt = best_nt;
        g.run_fpt = best_f;
    }
    if (e == hipSuccess) e = copy_all(false);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(save);
    shapes_changed(c);
    if (e != hipSuccess) {
        set_err(c, "fca_autotune: %s", hipGetErrorString(e));
        c->broken = true;
        return FCA_E_DEVICE;
    }
    return FCA_OK;
}

// ---------------------------------------------------------------- captured step
fca_status fca_graph_capture(fca_ctx* c, int32_t iters, int32_t with_reset, double* loglik, double* R_out,
                             void* v_out, void* x_out) {
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (iters < 0) { set_err(c, "iters < 0"); return FCA_E_ARG; }
    const void* outs[] = {loglik, R_out, v_out, x_out};
    for (const void* p : outs)
        if (p && !is_device_ptr(p)) {
            set_err(c, "fca_graph_capture: outputs must be device pointers");
            return FCA_E_ARG;
        }
    fca_status st = refresh_active(c);
    if (st != FCA_OK) return st;
    FCA_HIP(c, hipStreamSynchronize(c->stream));
    if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    const std::vector<Group>& groups = c->all_active ? c->groups : c->groups_act;
    const EmProblem* probs = c->all_active ? c->probs : c->probs_act;
    if (!c->cap_stream) FCA_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    st = ensure_side_streams(c, (int)groups.size() - 1);
    if (st != FCA_OK) return st;
    const hipStream_t s = c->cap_stream;
    FCA_HIP(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    auto body = [&]() -> fca_status {
        if (with_reset) {
            fca_status r = restore_all(c, s);
            if (r != FCA_OK) return r;
        }
        int done = 0;
        do {
            const int chunk = iters == 0 ? 0 : std::min(kLChunk, iters - done);
            const int rows = chunk > 0 ? chunk : 1;
            fca_status r = enqueue_em_groups(c, groups, probs, chunk, done, false, s);
            if (r == FCA_OK && loglik) r = enqueue_ll_out(c, rows, iters > 0 ? iters : 1, done, loglik, s);
            if (r != FCA_OK) return r;
            c->graph_rows = rows;
            done += chunk;
        } while (done < iters);
        fca_status r = FCA_OK;
        if (R_out) r = enqueue_R_out(c, reinterpret_cast<double2*>(R_out), s, x_out != nullptr);
        if (r == FCA_OK && v_out) r = enqueue_v_out(c, v_out, s);
        if (r == FCA_OK && x_out) r = enqueue_separate(c, x_out, s, R_out != nullptr);
        return r;
    };
    st = body();
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (st != FCA_OK || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (st == FCA_OK) {
            set_err(c, "fca_graph_capture: hipStreamEndCapture: %s", hipGetErrorString(ee));
            st = FCA_E_DEVICE;
        }
        c->broken = false;  // nothing ran; the context's state is unchanged
        (void)hipGetLastError();
        return st;
    }
    c->graph = g;
    FCA_HIP(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    c->graph_version = c->shape_version;
    return FCA_OK;
}

fca_status fca_graph_launch(fca_ctx* c, int32_t count) {
    if (!c) return FCA_E_ARG;
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (!c->gexec) { set_err(c, "fca_graph_launch: nothing captured"); return FCA_E_STATE; }
    if (c->act_dirty || c->graph_version != c->shape_version) {
        set_err(c, "fca_graph_launch: active mixtures or launch shapes changed since the capture");
        return FCA_E_STATE;
    }
    if (count < 1) { set_err(c, "fca_graph_launch: count < 1"); return FCA_E_ARG; }
    for (int i = 0; i < count; ++i) FCA_HIP(c, hipGraphLaunch(c->gexec, c->stream));
    c->last_rows = c->graph_rows;
    c->last_active = c->active;
    return check_flags(c);
}

fca_status fca_loglik_per_freq(const fca_ctx* cc, int32_t rows, double* ll_out) {
    if (!cc || !ll_out) return FCA_E_ARG;
    fca_ctx* c = const_cast<fca_ctx*>(cc);
    if (c->broken) { set_err(c, "context unusable after an earlier device error"); return FCA_E_STATE; }
    if (c->last_rows == 0) { set_err(c, "fca_loglik_per_freq: no EM call yet"); return FCA_E_STATE; }
    if (rows < 1 || rows > c->last_rows) {
        set_err(c, "fca_loglik_per_freq: rows %d outside 1..%d", rows, c->last_rows);
        return FCA_E_ARG;
    }
    const hipStream_t s = c->stream;
    const int64_t n = (int64_t)rows * c->nprob;
    FCA_HIP(c, hipMemcpyAsync(ll_out, c->ll + (int64_t)(c->last_rows - rows) * c->nprob, n * sizeof(double),
                              hipMemcpyDefault, s));
    const bool dev = is_device_ptr(ll_out);
    if (dev) {
        // NaN rows of the mixtures inactive in that call, one launch (the
        // list staged like the launch tables)
        FCA_HIP(c, hipEventSynchronize(c->table_ev));
        int ni = 0;
        for (int b = 0; b < c->B; ++b)
            if (!c->last_active[b]) c->inactive_host[ni++] = b;
        if (ni) {
            FCA_HIP(c, hipMemcpyAsync(c->inactive_dev, c->inactive_host, (size_t)ni * sizeof(int),
                                      hipMemcpyHostToDevice, s));
            FCA_HIP(c, launch_nan_rows(ll_out, c->nprob, rows, c->F, c->F, c->inactive_dev, ni, s));
            // the same list as the last table rebuild's unless the activity
            // changed since, which marks the tables for a rebuild anyway
            FCA_HIP(c, hipEventRecord(c->table_ev, s));
        }
        FCA_HIP(c, hipStreamSynchronize(s));
        return FCA_OK;
    }
    FCA_HIP(c, hipStreamSynchronize(s));
    for (int b = 0; b < c->B; ++b) {
        if (c->last_active[b]) continue;
        for (int r = 0; r < rows; ++r) {
            double* row = ll_out + (int64_t)r * c->nprob + (int64_t)b * c->F;
            for (int f = 0; f < c->F; ++f) row[f] = std::numeric_limits<double>::quiet_NaN();
        }
    }
    return FCA_OK;
}

}  // extern "C"
