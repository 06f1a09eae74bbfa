// C-ABI front end for many independent streams processed in shared passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/erx.h"
#include "erx_internal.h"
#include "erx_runtime.h"

using namespace erx;

#define fail erx::set_error
#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(ERX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr int NSLOT = 2;  // descriptor upload slots (double buffered)

struct BStream {
    int b = 0, p = 0, NT = 0;
    float alpha = 0.f;
    long long t = 0;
    void* state = nullptr;  // FP64, or FP32 with state_fp32
    float* scores = nullptr;
    float* scores_n = nullptr;
    long long cap_lines = 0;
    int last_n = 0;
};

struct Group {
    int NT = 0;
    bool vecable = false;       // every stream of the group has a band count divisible by 4
    hipStream_t gs = nullptr;   // the group's stream: groups run concurrently within a push
    hipEvent_t done_ev = nullptr;
    long long E = 0;
    std::vector<int> streams;  // longest work first
    void* stats = nullptr;  // FP64, or FP32 with state_fp32
    void* carry = nullptr;
    float* Mt = nullptr;
    float* mu32 = nullptr;
    float* mscale = nullptr;
    int* gredo = nullptr;
    int* flags = nullptr;
    float* cond = nullptr;
    StreamDesc* d_sd[NSLOT] = {nullptr, nullptr};
    StreamDesc* h_sd[NSLOT] = {nullptr, nullptr};  // pinned
    hipEvent_t slot_ev[NSLOT] = {nullptr, nullptr};
    int next_slot = 0;
    // graphs keyed by (slot, nstreams, nlines, nseg, pmax)
    std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;  // (slot, nsd, L, S, pmax, vec4)
};

size_t esize(int dtype) { return dtype == ERX_F32 ? 4 : 2; }

}  // namespace

struct erx_batch {
    erx_config cfg;
    std::vector<BStream> st;
    std::vector<Group> groups;
    hipStream_t stream = nullptr;      // the library's own non-blocking stream: all work runs here
    hipStream_t user = nullptr;        // the caller's stream (ordered with events)
    bool has_user = false;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipEvent_t fork_ev = nullptr;      // the push's start, which every group stream waits for
    hipStream_t own_stream = nullptr;
    unsigned long long* ctr = nullptr;
    bool use_graphs = true;
    int small_mode = -1;  // fused path for one-tile streams: -1 auto, 0 off, 1 on, 2 on (streamed variant)
    unsigned long long notpd_before = 0;
};

namespace {

void destroy_all(erx_batch* bt)
{
    if (bt->stream) (void)hipStreamSynchronize(bt->stream);
    for (auto& g : bt->groups) {
        void* d[] = {g.stats, g.carry, g.Mt, g.mu32, g.mscale, g.gredo, g.flags, g.cond, g.d_sd[0], g.d_sd[1]};
        for (void* p : d)
            if (p) (void)hipFree(p);
        for (int k = 0; k < NSLOT; ++k) {
            if (g.h_sd[k]) (void)hipHostFree(g.h_sd[k]);
            if (g.slot_ev[k]) (void)hipEventDestroy(g.slot_ev[k]);
        }
        for (auto& kv : g.graphs) (void)hipGraphExecDestroy(kv.second);
        if (g.gs) (void)hipStreamSynchronize(g.gs);
        if (g.done_ev) (void)hipEventDestroy(g.done_ev);
        if (g.gs) (void)hipStreamDestroy(g.gs);
    }
    for (auto& s : bt->st) {
        if (s.state) (void)hipFree(s.state);
        if (s.scores) (void)hipFree(s.scores);
        if (s.scores_n) (void)hipFree(s.scores_n);
    }
    if (bt->ctr) (void)hipFree(bt->ctr);
    if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
    if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
    if (bt->fork_ev) (void)hipEventDestroy(bt->fork_ev);
    if (bt->own_stream) (void)hipStreamDestroy(bt->own_stream);
}

bool device_ptr(const void* ptr)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

long long packed_offset(int r, int c, int NT)
{
    const int I = r >> 4, J = c >> 4, rr = r & 15, cc = c & 15;
    const long long u = (long long)I * NT - (long long)I * (I - 1) / 2 + (J - I);
    return u * 256 + (16 * (rr >> 2) + cc) * 4 + (rr & 3);
}

}  // namespace

extern "C" {

erx_batch* erx_batch_create(int nstreams, const int* bands, const int* pixels, const float* momentum,
                            const erx_config* common)
{
    if (nstreams < 1 || !bands || !pixels || !momentum || !common) {
        fail(ERX_EINVAL, "erx_batch_create: need nstreams >= 1 and non-NULL arrays and config");
        return nullptr;
    }
    const erx_config& c = *common;
    if (!(c.ridge >= 0.0f) || !std::isfinite(c.ridge) || (c.dtype != ERX_F32 && c.dtype != ERX_F16 && c.dtype != ERX_U16) ||
        c.precision < ERX_GRAM_FP32 || c.precision > ERX_GRAM_SPLIT16 || !(c.fp64_cond_threshold >= 0.0) || c.block_lines < 1 || c.scan_lines < 1 ||
        c.cond_estimate < -1 || c.cond_estimate > 1 || (c.normalise != 0 && c.normalise != 1) ||
        (c.score_arith != ERX_SCORE_SPLIT16 && c.score_arith != ERX_SCORE_FP32) || c.srp_dims != 0 ||
        c.background != ERX_BG_EMA || (c.state_fp32 != 0 && c.state_fp32 != 1) || c.score_tiles < 0 ||
        c.score_tiles > 2 || (c.gram_macro != 0 && c.gram_macro != 64 && c.gram_macro != 128)) {
        fail(ERX_EINVAL, "erx_batch_create: invalid common configuration");
        return nullptr;
    }
    for (int s = 0; s < nstreams; ++s) {
        if (bands[s] < 1 || bands[s] > ERX_MAX_BANDS || pixels[s] < 2 || !(momentum[s] > 0.f && momentum[s] <= 1.f)) {
            fail(ERX_EINVAL, "stream %d: bands in [1, %d], pixels >= 2 and momentum in (0, 1] required", s,
                 ERX_MAX_BANDS);
            return nullptr;
        }
    }
    erx_batch* bt = new (std::nothrow) erx_batch();
    if (!bt) {
        fail(ERX_ENOMEM, "out of host memory");
        return nullptr;
    }
    bt->cfg = c;
    bt->st.resize(nstreams);
    // streams are grouped by tile count and by whether 4-band vector loads apply (a pass
    // takes them only when all its streams allow them)
    std::map<std::pair<int, int>, std::vector<int>> byNT;
    for (int s = 0; s < nstreams; ++s) {
        BStream& S = bt->st[s];
        S.b = bands[s];
        S.p = pixels[s];
        S.NT = (S.b + 15) / 16;
        S.alpha = momentum[s];
        byNT[{S.NT, S.b % 4 == 0 ? 1 : 0}].push_back(s);
    }
    bool ok = hipStreamCreateWithFlags(&bt->own_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&bt->fork_ev, hipEventDisableTiming) == hipSuccess;
    bt->stream = bt->own_stream;
    ok = ok && hipMalloc(&bt->ctr, 4 * sizeof(unsigned long long)) == hipSuccess &&
         hipMemset(bt->ctr, 0, 4 * sizeof(unsigned long long)) == hipSuccess;
    const size_t C = (size_t)c.block_lines;
    const size_t ss = c.state_fp32 ? sizeof(float) : sizeof(double);
    for (auto& kv : byNT) {
        if (!ok) break;
        Group g;
        g.NT = kv.first.first;
        g.vecable = kv.first.second != 0;
        g.E = stat_entries(g.NT);
        g.streams = kv.second;
        std::stable_sort(g.streams.begin(), g.streams.end(), [&](int a, int b2) {
            const BStream &A = bt->st[a], &B = bt->st[b2];
            return (double)A.p * A.b * A.b > (double)B.p * B.b * B.b;
        });
        const size_t ns = g.streams.size();
        const size_t nseg_max = C / c.scan_lines + ns + 1;
        const size_t NTL = (size_t)g.NT * (g.NT + 1) / 2;
        ok = ok && hipMalloc(&g.stats, C * g.E * ss) == hipSuccess &&
             hipMalloc(&g.carry, nseg_max * g.E * ss) == hipSuccess &&
             hipMalloc(&g.Mt, C * NTL * 256 * sizeof(float)) == hipSuccess &&
             hipMalloc(&g.mu32, C * 16 * g.NT * sizeof(float)) == hipSuccess &&
             hipMalloc(&g.mscale, C * sizeof(float)) == hipSuccess &&
             hipMalloc(&g.gredo, C * GRAM_MACROS_MAX * sizeof(int)) == hipSuccess &&
             hipMalloc(&g.flags, C * sizeof(int)) == hipSuccess && hipMalloc(&g.cond, C * sizeof(float)) == hipSuccess;
        ok = ok && hipStreamCreateWithFlags(&g.gs, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&g.done_ev, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; k < NSLOT && ok; ++k)
            ok = hipMalloc(&g.d_sd[k], ns * sizeof(StreamDesc)) == hipSuccess &&
                 hipHostMalloc(&g.h_sd[k], ns * sizeof(StreamDesc), hipHostMallocDefault) == hipSuccess &&
                 hipEventCreateWithFlags(&g.slot_ev[k], hipEventDisableTiming) == hipSuccess;
        for (int s : g.streams) {
            if (!ok) break;
            ok = hipMalloc(&bt->st[s].state, g.E * ss) == hipSuccess &&
                 hipMemset(bt->st[s].state, 0, g.E * ss) == hipSuccess;
        }
        bt->groups.push_back(g);
    }
    if (!ok) {
        (void)hipGetLastError();
        destroy_all(bt);
        delete bt;
        fail(ERX_ENOMEM, "erx_batch_create: device allocation failed");
        return nullptr;
    }
    return bt;
}

int erx_batch_set_stream(erx_batch* bt, void* s)
{
    if (!bt) return fail(ERX_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(bt->stream));
    bt->user = (hipStream_t)s;
    bt->has_user = true;
    return ERX_OK;
}

int erx_batch_use_graphs(erx_batch* bt, int on)
{
    if (!bt) return fail(ERX_EINVAL, "NULL batch");
    bt->use_graphs = on != 0;
    return ERX_OK;
}

int erx_batch_small_path(erx_batch* bt, int mode)
{
    if (!bt) return fail(ERX_EINVAL, "NULL batch");
    if (mode < -1 || mode > 2) return fail(ERX_EINVAL, "small-path mode must be -1, 0, 1 or 2");
    bt->small_mode = mode;
    return ERX_OK;
}

int erx_batch_push(erx_batch* bt, const void* const* lines, const int* nlines)
{
    if (!bt || !lines || !nlines) return fail(ERX_EINVAL, "NULL argument");
    const erx_config& c = bt->cfg;
    const int ns = (int)bt->st.size();
    const size_t esz = esize(c.dtype);
    for (int s = 0; s < ns; ++s) {
        if (nlines[s] < 0) return fail(ERX_EINVAL, "stream %d: negative line count", s);
        if (nlines[s] == 0) continue;
        if (!lines[s] || !device_ptr(lines[s]))
            return fail(ERX_EINVAL, "stream %d: the line buffer must be device memory", s);
        if (((uintptr_t)lines[s] % esz) != 0)
            return fail(ERX_EINVAL, "stream %d: line buffer must be aligned to its element size", s);
    }
    // result buffers
    for (int s = 0; s < ns; ++s) {
        BStream& S = bt->st[s];
        if (nlines[s] > S.cap_lines) {
            HIPCHK(hipStreamSynchronize(bt->stream));
            if (S.scores) (void)hipFree(S.scores);
            if (S.scores_n) (void)hipFree(S.scores_n);
            S.scores = S.scores_n = nullptr;
            S.cap_lines = 0;
            if (hipMalloc(&S.scores, (size_t)nlines[s] * S.p * sizeof(float)) != hipSuccess ||
                (c.normalise && hipMalloc(&S.scores_n, (size_t)nlines[s] * S.p * sizeof(float)) != hipSuccess)) {
                (void)hipGetLastError();
                return fail(ERX_ENOMEM, "stream %d: cannot allocate the score buffer", s);
            }
            S.cap_lines = nlines[s];
        }
        S.last_n = nlines[s];
    }
    unsigned long long cnt[4];
    HIPCHK(hipMemcpyAsync(cnt, bt->ctr, sizeof cnt, hipMemcpyDeviceToHost, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    bt->notpd_before = cnt[1];
    // the caller's earlier work (which produced the lines) comes first
    if (bt->has_user) {
        HIPCHK(hipEventRecord(bt->ev_in, bt->user));
        HIPCHK(hipStreamWaitEvent(bt->stream, bt->ev_in, 0));
    }

    const double thr = c.fp64_cond_threshold;
    const bool decides = thr > 0.0 && !std::isinf(thr);
    const int want_cond = c.cond_estimate == 1 || (c.cond_estimate == -1 && decides) ? 1 : 0;
    const bool fp64_pass = !std::isinf(thr);
    const int C = c.block_lines, seg = c.scan_lines;

    // every group runs on its own stream from the push's start (fork) and the push ends when
    // all of them have (join): groups of different tile counts overlap on the device
    // The host deals one pass to each group in turn, so that every group has work queued
    // while it waits for a descriptor slot of another.
    HIPCHK(hipEventRecord(bt->fork_ev, bt->stream));
    const size_t ng = bt->groups.size();
    std::vector<std::vector<int>> offs(ng);
    std::vector<char> live(ng, 1);
    for (size_t gi = 0; gi < ng; ++gi) {
        HIPCHK(hipStreamWaitEvent(bt->groups[gi].gs, bt->fork_ev, 0));
        offs[gi].assign(bt->groups[gi].streams.size(), 0);
    }
    for (bool any = true; any;) {
        any = false;
        for (size_t gi = 0; gi < ng; ++gi) {
            if (!live[gi]) continue;
            Group& g = bt->groups[gi];
            hipStream_t gstream = g.gs;
            // (the fused kernels keep an FP64 state: with FP32 storage every group takes the general path)
            if (g.NT == 1 && !c.state_fp32 &&
                (bt->small_mode >= 1 || (bt->small_mode == -1 && g.streams.size() >= 32))) {
                // fused path: one launch, every stream's lines in order
                const int slot = g.next_slot;
                g.next_slot = (g.next_slot + 1) % NSLOT;
                HIPCHK(hipEventSynchronize(g.slot_ev[slot]));
                StreamDesc* hd = g.h_sd[slot];
                int nsd = 0, vec4 = 1, pmax = 0, lmax = 0, al16 = bt->small_mode != 2;
                for (int s : g.streams) {
                    if (nlines[s] == 0) continue;
                    BStream& B = bt->st[s];
                    StreamDesc d{};
                    d.x = lines[s];
                    d.out = B.scores;
                    d.outn = c.normalise ? B.scores_n : nullptr;
                    d.state = B.state;
                    d.t0 = B.t;
                    d.alpha = B.alpha;
                    d.eps = c.ridge;
                    d.p = B.p;
                    d.b = B.b;
                    d.n = nlines[s];
                    hd[nsd++] = d;
                    vec4 = vec4 && (B.b % 4 == 0) && ((uintptr_t)lines[s] % (4 * esz)) == 0;
                    pmax = std::max(pmax, B.p);
                    const long long lb = (long long)B.p * B.b * esz;  // bytes of one line
                    al16 = al16 && lb % 16 == 0 && (uintptr_t)lines[s] % 16 == 0;
                    lmax = (int)std::min<long long>(std::max<long long>(lmax, lb), 1LL << 30);
                    B.t += nlines[s];
                }
                if (nsd > 0) {
                    Pass P{};
                    P.sd = g.d_sd[slot];
                    P.nstreams = nsd;
                    P.pmax = pmax;
                    P.vec4 = vec4;
                    HIPCHK(hipMemcpyAsync(g.d_sd[slot], hd, nsd * sizeof(StreamDesc), hipMemcpyHostToDevice,
                                          gstream));
                    HIPCHK(launch_small(c.dtype, P, c.normalise, bt->ctr, al16 ? lmax : 0, gstream));
                }
                HIPCHK(hipEventRecord(g.slot_ev[slot], gstream));
                HIPCHK(hipEventRecord(g.done_ev, gstream));
                HIPCHK(hipStreamWaitEvent(bt->stream, g.done_ev, 0));
                live[gi] = 0;
                continue;
            }
            std::vector<int>& off = offs[gi];
            {
                // streams with lines left, longest work first
                std::vector<int> act;
                for (size_t k = 0; k < g.streams.size(); ++k)
                    if (off[k] < nlines[g.streams[k]]) act.push_back((int)k);
                if (act.empty()) {  // the group is done: the push's end waits for it
                    HIPCHK(hipEventRecord(g.done_ev, gstream));
                    HIPCHK(hipStreamWaitEvent(bt->stream, g.done_ev, 0));
                    live[gi] = 0;
                    continue;
                }
                any = true;
                int quota = C / (int)act.size();
                quota = quota >= seg ? (quota / seg) * seg : seg;
                // descriptors
                const int slot = g.next_slot;
                g.next_slot = (g.next_slot + 1) % NSLOT;
                HIPCHK(hipEventSynchronize(g.slot_ev[slot]));  // the slot's previous upload has run
                StreamDesc* hd = g.h_sd[slot];
                int L = 0, S = 0, nsd = 0, pmax = 0, vec4 = 1;
                std::vector<std::pair<int, int>> taken;  // (group index, lines)
                for (int k : act) {
                    const int s = g.streams[k];
                    const BStream& B = bt->st[s];
                    int kl = std::min(nlines[s] - off[k], quota);
                    if (L + kl > C) kl = C - L;
                    if (kl <= 0) break;
                    StreamDesc d{};
                    d.x = (const char*)lines[s] + (size_t)off[k] * B.p * B.b * esz;
                    d.out = B.scores + (size_t)off[k] * B.p;
                    d.outn = c.normalise ? B.scores_n + (size_t)off[k] * B.p : nullptr;
                    d.state = B.state;
                    d.t0 = B.t;
                    d.alpha = B.alpha;
                    d.eps = c.ridge;
                    d.p = B.p;
                    d.b = B.b;
                    d.n = kl;
                    d.line0 = L;
                    d.seg0 = S;
                    hd[nsd++] = d;
                    L += kl;
                    S += (kl + seg - 1) / seg;
                    pmax = std::max(pmax, B.p);
                    vec4 = vec4 && (B.b % 4 == 0) && ((uintptr_t)d.x % (4 * esz)) == 0;
                    taken.push_back({k, kl});
                }
                Pass P{};
                P.sd = g.d_sd[slot];
                P.nstreams = nsd;
                P.nlines = L;
                P.nseg = S;
                P.seg = seg;
                P.pmax = pmax;
                P.vec4 = vec4;
                P.mscale = g.mscale;
                P.gredo = g.gredo;
                P.sf32 = c.state_fp32;
                P.spt = c.score_tiles;
                P.gmacro = c.gram_macro;
                auto record = [&]() -> hipError_t {
                    hipError_t e = hipMemcpyAsync(g.d_sd[slot], hd, nsd * sizeof(StreamDesc), hipMemcpyHostToDevice,
                                                  gstream);
                    if (e != hipSuccess) return e;
                    return run_pass(gstream, P, g.NT, c.dtype, c.precision, c.score_arith, g.stats, g.carry, g.Mt, g.mu32, g.flags, g.cond, thr,
                                    want_cond, fp64_pass, c.normalise != 0, bt->ctr, nullptr);
                };
                if (bt->use_graphs) {
                    const auto key = std::make_tuple(slot, nsd, L, S, pmax, vec4);
                    auto it = g.graphs.find(key);
                    if (it == g.graphs.end()) {
                        hipGraph_t graph;
                        HIPCHK(hipStreamBeginCapture(gstream, hipStreamCaptureModeThreadLocal));
                        const hipError_t e = record();
                        hipGraph_t got = nullptr;
                        const hipError_t e2 = hipStreamEndCapture(gstream, &got);  // always ends the capture
                        if (e != hipSuccess || e2 != hipSuccess) {
                            if (got) (void)hipGraphDestroy(got);
                            return fail(ERX_EDEVICE, "graph capture failed: %s", hipGetErrorString(e ? e : e2));
                        }
                        graph = got;
                        hipGraphExec_t exec;
                        const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                        (void)hipGraphDestroy(graph);
                        if (e3 != hipSuccess) return fail(ERX_EDEVICE, "graph instantiation failed");
                        it = g.graphs.emplace(key, exec).first;
                    }
                    HIPCHK(hipGraphLaunch(it->second, gstream));
                } else {
                    HIPCHK(record());
                }
                HIPCHK(hipEventRecord(g.slot_ev[slot], gstream));
                for (auto& tk : taken) {
                    off[tk.first] += tk.second;
                    bt->st[g.streams[tk.first]].t += tk.second;
                }
            }
        }
    }
    // the caller's later work sees the scores
    if (bt->has_user) {
        HIPCHK(hipEventRecord(bt->ev_out, bt->stream));
        HIPCHK(hipStreamWaitEvent(bt->user, bt->ev_out, 0));
    }
    return ERX_OK;
}

int erx_batch_scores(erx_batch* bt, float* const* out)
{
    if (!bt || !out) return fail(ERX_EINVAL, "NULL argument");
    for (size_t s = 0; s < bt->st.size(); ++s) {
        const BStream& B = bt->st[s];
        if (B.last_n == 0 || !out[s]) continue;  // a NULL buffer skips the stream
        HIPCHK(hipMemcpyAsync(out[s], B.scores, (size_t)B.last_n * B.p * sizeof(float), hipMemcpyDefault,
                              bt->stream));
    }
    unsigned long long cnt[4];
    HIPCHK(hipMemcpyAsync(cnt, bt->ctr, sizeof cnt, hipMemcpyDeviceToHost, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    if (cnt[1] > bt->notpd_before)
        return fail(ERX_ENOTPD, "at least one line had a covariance that is not positive definite");
    return ERX_OK;
}

int erx_batch_get_state(erx_batch* bt, int stream, long long* t, double* mu, double* K)
{
    if (!bt || stream < 0 || stream >= (int)bt->st.size()) return fail(ERX_EINVAL, "bad batch or stream index");
    const BStream& B = bt->st[stream];
    const long long E = stat_entries(B.NT);
    std::vector<double> s(E);
    if (bt->cfg.state_fp32) {
        std::vector<float> f(E);
        HIPCHK(hipMemcpyAsync(f.data(), B.state, E * sizeof(float), hipMemcpyDeviceToHost, bt->stream));
        HIPCHK(hipStreamSynchronize(bt->stream));
        for (long long i = 0; i < E; ++i) s[i] = f[i];
    } else {
        HIPCHK(hipMemcpyAsync(s.data(), B.state, E * sizeof(double), hipMemcpyDeviceToHost, bt->stream));
        HIPCHK(hipStreamSynchronize(bt->stream));
    }
    const int NTL = B.NT * (B.NT + 1) / 2;
    if (t) *t = B.t;
    if (mu)
        for (int j = 0; j < B.b; ++j) mu[j] = s[(size_t)NTL * 256 + j];
    if (K)
        for (int r = 0; r < B.b; ++r)
            for (int c2 = 0; c2 < B.b; ++c2)
                K[(size_t)r * B.b + c2] = (r <= c2) ? s[packed_offset(r, c2, B.NT)] : s[packed_offset(c2, r, B.NT)];
    return ERX_OK;
}

int erx_batch_stats(erx_batch* bt, erx_stats_t* out)
{
    if (!bt || !out) return fail(ERX_EINVAL, "NULL argument");
    unsigned long long c[4];
    HIPCHK(hipMemcpyAsync(c, bt->ctr, sizeof c, hipMemcpyDeviceToHost, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    long long lines = 0;
    for (auto& s : bt->st) lines += s.t;
    out->lines = lines;
    out->fp64_refactors = (long long)c[0];
    out->notpd = (long long)c[1];
    float mc;
    const unsigned int bits = (unsigned int)(c[2] & 0xffffffffull);
    std::memcpy(&mc, &bits, sizeof mc);
    out->max_cond = mc;
    return ERX_OK;
}

int erx_batch_synchronize(erx_batch* bt)
{
    if (!bt) return fail(ERX_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(bt->stream));
    return ERX_OK;
}

void erx_batch_destroy(erx_batch* bt)
{
    if (!bt) return;
    destroy_all(bt);
    delete bt;
}

}  // extern "C"
