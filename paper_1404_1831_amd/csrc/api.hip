// Host side of libfbpq: the C ABI of include/fbpq.h. Index upload and
// validation, the index file reader, the table build, and the search
// pipeline: half keys -> sorted prefixes -> traversal -> layout -> scan+top-k,
// with a second round for the queries whose traversal needs a longer sorted
// prefix or more visited cells than the first round provided.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "fbpq.h"
#include "fbpq_dev.h"

using namespace fbpq;

static constexpr size_t kScanLdsLimit = 74 * 1024;  // two scan workgroups per CU (160 KB LDS)

// Scratch of the no-allocation search (fbpq_search_device_noalloc): one copy
// per device, resident while the process lives. Host code never uses the
// array's name as an address; it looks up each device's copy once with
// hipGetSymbolAddress and passes that pointer on.
static constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

}  // namespace

struct fbpq_index {
    int device = 0;
    bool shared = false;  // a serving lane: index arrays belong to another handle
    bool poisoned = false;
    int64_t inject_after = 0;  // option "inject_device_error": countdown to a reported failure
    bool tables = false;
    DevIndex dv{};
    hipStream_t stream = nullptr;
    hipStream_t cur = nullptr;  // stream of the search in progress (workspace growth is ordered on it)
    // second stream: the query tables of a round run on it beside the first
    // layer and the traversal, forked and joined through two events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;  // the two-pass scans beside the cell scan
    // owned device allocations
    float *C1 = nullptr, *C2 = nullptr, *R = nullptr;
    float *QL = nullptr, *SL = nullptr;  // local codebooks (HBPQ), or null
    float *Rot = nullptr;                // OPQ rotation, or null
    int64_t *offsets = nullptr;
    uint8_t *codesA = nullptr, *codesB = nullptr;
    uint32_t *ids = nullptr;
    float *CR1 = nullptr, *CR2 = nullptr, *nR = nullptr, *nC1 = nullptr, *nC2 = nullptr;
    _Float16 *Cs1 = nullptr, *Cs2 = nullptr;  // two-part FP16 half-centroids (D/2 = 64)
    float csc1 = 1.f, csc2 = 1.f;
    bool split_keys = true;  // option "split_keys": approximate keys from the FP16 parts
    size_t base_bytes = 0, table_bytes = 0;
    // workspace, grown on demand: slots [0, 48) for the first round of a
    // search (the round a graph captures), [48, 96) for its retry rounds
    DevBuf ws[96];
    int ws_base = 0;
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    // no-allocation searches: workspace carved from the device's static scratch
    // array for the duration of one call, host staging in pageable memory
    struct Arena {
        unsigned char *base = nullptr;  // this device's scratch array (device address)
        size_t cap = 0, used = 0;
        void *slot[96] = {};
        size_t bytes[96] = {};
    } arena;
    bool use_arena = false;
    std::vector<char> host_stage;
    // the last fbpq_search_device_async, while its retry rounds (if any) are
    // still to run: finished by fbpq_search_device_finish or the next search
    bool async_open = false;
    hipEvent_t async_ev = nullptr;      // recorded after its first round
    int32_t *async_count = nullptr;     // pinned: queries its first round left over
    struct AsyncState {
        const float *d_q;
        int64_t nq;
        int32_t P;
        int64_t max_cells, lcap;
        int32_t k_max;
        int64_t *d_ids;
        float *d_d;
        hipStream_t st;
    } async{};
    // profiler: events recorded around launches while `profile` is on
    bool profile = false;
    int64_t prof_mask = -1;  // stages timed while profiling
    struct Ev {
        hipEvent_t a, b;
        int stage;
    };
    std::vector<Ev> ev_live;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[FBPQ_NUM_STAGES] = {0};
    int64_t prof_n[FBPQ_NUM_STAGES] = {0};
    // options
    int32_t prefix = 128;
    int32_t prefix_cap = kMaxPrefix;  // longest prefix a retry round may take
    int64_t max_cells = 4096;
    int32_t chunk = 8192;
    bool items = true;
    bool hint_first = true;  // without graph replay: a batch whose budget classes all retried before starts deeper
    bool persist = false;   // cell scan as a persistent kernel over a device work queue
    int32_t tile = 8192;    // candidates per work item of the persistent scan
    int32_t pwaves = 4;     // wavefronts per workgroup of the persistent scan
    int32_t block_min = 2;  // the wave prefix select samples the key kernel's block minima: 0 off, 1 on, 2 when T >= 4096
    int32_t pop_budget = 512;  // cells popped one at a time before the threshold kernel takes over
    // per floor(log2(min(L, N))): the prefix length at which retried queries of
    // that budget last succeeded; retry rounds start there instead of at 4P
    int32_t p_hint[64] = {0};
    int64_t c_hint[64] = {0};  // ... and the visited cells they needed
    // path counters (option "stats")
    unsigned long long *stats_dev = nullptr;
    int64_t stat_retried = 0;
    // captured first round (option "graph"): replayed while its key matches
    bool graph = false;
    int64_t ws_gen = 0;  // bumped whenever a workspace buffer moves
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const float *d_q;
        int64_t nq, lcap, max_cells, ws_gen;
        int64_t *d_ids;
        float *d_d;
        int32_t k_max, P, chunk, pop_budget;
        bool items;
        int32_t block_min;
        bool persist;
        int32_t tile, pwaves;
        unsigned long long *stats;
        bool split;
        bool operator==(const GraphKey &o) const
        {
            return d_q == o.d_q && nq == o.nq && lcap == o.lcap && max_cells == o.max_cells &&
                   ws_gen == o.ws_gen && d_ids == o.d_ids && d_d == o.d_d && k_max == o.k_max && P == o.P &&
                   chunk == o.chunk && pop_budget == o.pop_budget && items == o.items &&
                   block_min == o.block_min && persist == o.persist && tile == o.tile && pwaves == o.pwaves &&
                   stats == o.stats && split == o.split;
        }
    } gkey{};
    int64_t graph_replays = 0;
};

namespace {

enum WsSlot {
    W_Q, W_KEYS, W_LKEY, W_LIDX, W_HDR, W_W, W_ROWNE, W_ROWCAND, W_COLNE, W_COLTOT, W_NECS,
    W_NECNT, W_NEBEG, W_NECST, W_CMCELL, W_CMPRE, W_L, W_K, W_QLIST, W_FAIL, W_IDS, W_D,
    W_DBGAB, W_DBGTAKE, W_DBGBEG, W_DBGPOS, W_DBGD, W_SPLIT, W_NESLOT, W_SLOTIJ, W_COUNTER,
    W_LQ, W_ITEMN, W_PSTAT, W_SELDONE, W_QROT, W_PSORT, W_BIG, W_LAYSCR, W_KMIN, W_PITEMS, W_PCTL,
    W_PQNIT, W_PQDONE, W_NSLOTS
};
constexpr int kWsSet = 48;  // slots per workspace set
static_assert(W_NSLOTS <= kWsSet, "workspace slots");

// a failure injected by the option "inject_device_error" (tests of error handling)
#define HCK_INJECTED(ix) ((ix)->inject_after > 0 && --(ix)->inject_after == 0)
#define HCK(ix, expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = HCK_INJECTED(ix) ? hipErrorLaunchFailure : (expr);                       \
        if (e_ != hipSuccess) {                                                                 \
            (ix)->poisoned = true;                                                              \
            return fail(FBPQ_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
        }                                                                                       \
    } while (0)

// Workspace buffers grow with stream-ordered frees and allocations on the
// stream of the search in progress, so that growing one lane's buffer never
// waits for the work of other streams (hipFree would synchronize the device).
int ws_get(fbpq_index *ix, int slot, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 8;
    if (ix->use_arena) {
        fbpq_index::Arena &ar = ix->arena;
        const int i = slot + ix->ws_base;
        if (!ar.slot[i] || ar.bytes[i] < bytes) {
            const size_t at = (ar.used + 255) & ~(size_t)255;
            if (at > ar.cap || bytes > ar.cap - at)
                return fail(FBPQ_E_CAPACITY, "the search needs more than the %zu bytes of no-allocation scratch",
                            ar.cap);
            ar.slot[i] = ar.base + at;
            ar.bytes[i] = bytes;
            ar.used = at + bytes;
        }
        *out = ar.slot[i];
        return FBPQ_OK;
    }
    DevBuf &b = ix->ws[slot + ix->ws_base];
    if (b.cap < bytes) {
        hipStream_t st = ix->cur ? ix->cur : ix->stream;
        if (b.p) {
            HCK(ix, hipFreeAsync(b.p, st));
            b.p = nullptr;
            b.cap = 0;
        }
        const size_t nb = std::max(bytes, b.cap + b.cap / 2);
        if (ix->ws_base == 0) ++ix->ws_gen;  // a buffer a captured round may use moved
        hipError_t e = hipMallocAsync(&b.p, nb, st);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(FBPQ_E_OOM, "device allocation of %zu bytes failed", nb);
        }
        b.cap = nb;
    }
    *out = b.p;
    return FBPQ_OK;
}

// Buffer of a workspace slot obtained earlier in this search.
void *ws_ptr(fbpq_index *ix, int slot)
{
    return ix->use_arena ? ix->arena.slot[slot + ix->ws_base] : ix->ws[slot + ix->ws_base].p;
}

int pinned_get(fbpq_index *ix, size_t bytes, void **out)
{
    if (ix->use_arena) {  // no-allocation searches stage through pageable host memory
        if (ix->host_stage.size() < bytes) ix->host_stage.resize(std::max<size_t>(bytes, 4096));
        *out = ix->host_stage.data();
        return FBPQ_OK;
    }
    if (ix->pinned_cap < bytes) {
        if (ix->pinned) {
            HCK(ix, hipStreamSynchronize(ix->stream));
            HCK(ix, hipHostFree(ix->pinned));
            ix->pinned = nullptr;
            ix->pinned_cap = 0;
        }
        const size_t nb = std::max(bytes, (size_t)1 << 16);
        if (hipHostMalloc(&ix->pinned, nb, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ix->pinned = nullptr;
            return fail(FBPQ_E_OOM, "pinned host allocation of %zu bytes failed", nb);
        }
        ix->pinned_cap = nb;
    }
    *out = ix->pinned;
    return FBPQ_OK;
}

hipEvent_t ev_take(fbpq_index *ix)
{
    if (!ix->ev_pool.empty()) {
        hipEvent_t e = ix->ev_pool.back();
        ix->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Wraps one kernel launch: events before and after it on `st` when profiling.
template <typename F>
hipError_t timed(fbpq_index *ix, int stage, hipStream_t st, F &&launch)
{
    if (!ix->profile || ix->use_arena || !((ix->prof_mask >> stage) & 1)) return launch();
    hipEvent_t a = ev_take(ix), b = ev_take(ix);
    if (a) (void)hipEventRecord(a, st);
    const hipError_t e = launch();
    if (b) (void)hipEventRecord(b, st);
    if (a && b) ix->ev_live.push_back({a, b, stage});
    return e;
}

// After the stream has been synchronized: fold the recorded intervals into the totals.
void prof_collect(fbpq_index *ix)
{
    for (auto &e : ix->ev_live) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            ix->prof_ms[e.stage] += ms;
            ix->prof_n[e.stage] += 1;
        } else {
            (void)hipGetLastError();
        }
        ix->ev_pool.push_back(e.a);
        ix->ev_pool.push_back(e.b);
    }
    ix->ev_live.clear();
}

std::mutex g_scratch_mu;
void *g_scratch_dev[64] = {};  // device address of each device's scratch array

// The device address of `scratch` on `device`, which must be current; looked
// up on the first call for each device and kept.
int scratch_addr(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= 64) return fail(FBPQ_E_DEVICE, "device %d out of range", device);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(FBPQ_E_DEVICE, "address of the scratch array on device %d: %s", device,
                        hipGetErrorString(e));
        }
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return FBPQ_OK;
}

int check_desc(const fbpq_index_desc *d)
{
    if (!d) return fail(FBPQ_E_INVALID, "null descriptor");
    if (d->D <= 0 || d->D % 2 || d->M <= 0 || d->M % 2 || d->D % d->M)
        return fail(FBPQ_E_FORMAT, "bad geometry D=%d M=%d (need D, M even and M | D)", d->D, d->M);
    const int mh = d->M / 2;
    if (!(mh == 1 || mh == 2 || mh == 4 || mh == 8 || mh == 16))
        return fail(FBPQ_E_FORMAT, "M=%d not supported (M/2 must be 1, 2, 4, 8 or 16)", d->M);
    if (d->Kc != FBPQ_KC) return fail(FBPQ_E_FORMAT, "Kc=%d, only 256 is supported", d->Kc);
    if (d->T <= 0 || d->T > (1 << 20)) return fail(FBPQ_E_FORMAT, "bad T=%d", d->T);
    if (d->N < 0 || d->N > (int64_t)0xffffffffLL) return fail(FBPQ_E_FORMAT, "bad N=%lld", (long long)d->N);
    if (d->D > 4096) return fail(FBPQ_E_FORMAT, "D=%d too large", d->D);
    if (!d->C1 || !d->C2 || !d->R || !d->offsets || (d->N > 0 && (!d->codes || !d->ids)))
        return fail(FBPQ_E_INVALID, "null array in descriptor");
    if ((d->QL == nullptr) != (d->SL == nullptr))
        return fail(FBPQ_E_INVALID, "local codebooks need both QL and SL");
    if (d->Rot && d->D > 1024) return fail(FBPQ_E_INVALID, "an OPQ rotation needs D <= 1024");
    const int64_t C = (int64_t)d->T * d->T;
    if (d->offsets[0] != 0 || d->offsets[C] != d->N)
        return fail(FBPQ_E_FORMAT, "offsets must start at 0 and end at N");
    for (int64_t c = 0; c < C; ++c)
        if (d->offsets[c + 1] < d->offsets[c])
            return fail(FBPQ_E_FORMAT, "offsets decrease at cell %lld", (long long)c);
    return FBPQ_OK;
}

template <typename T>
int upload(fbpq_index *ix, T **dst, const void *src, size_t bytes)
{
    if (hipMalloc((void **)dst, bytes ? bytes : 8) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(FBPQ_E_OOM, "device allocation of %zu bytes failed", bytes);
    }
    ix->base_bytes += bytes;
    if (bytes) HCK(ix, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return FBPQ_OK;
}

void free_all(fbpq_index *ix)
{
    if (!ix) return;
    (void)hipSetDevice(ix->device);
    if (ix->stream) (void)hipStreamSynchronize(ix->stream);
    if (ix->side) (void)hipStreamSynchronize(ix->side);
    void *ps[] = {ix->C1, ix->C2, ix->R, ix->offsets, ix->codesA, ix->codesB, ix->ids,
                  ix->CR1, ix->CR2, ix->nR, ix->nC1, ix->nC2, ix->QL, ix->SL, ix->Rot, ix->Cs1, ix->Cs2};
    if (!ix->shared)
        for (void *p : ps)
            if (p) (void)hipFree(p);
    if (ix->stats_dev) (void)hipFree(ix->stats_dev);
    for (auto &b : ix->ws)
        if (b.p) (void)hipFree(b.p);
    if (ix->pinned) (void)hipHostFree(ix->pinned);
    if (ix->async_count) (void)hipHostFree(ix->async_count);
    if (ix->async_ev) (void)hipEventDestroy(ix->async_ev);
    for (auto &e : ix->ev_live) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto e : ix->ev_pool) (void)hipEventDestroy(e);
    if (ix->gexec) (void)hipGraphExecDestroy(ix->gexec);
    if (ix->side) {
        (void)hipStreamSynchronize(ix->side);
        (void)hipStreamDestroy(ix->side);
    }
    if (ix->ev_fork) (void)hipEventDestroy(ix->ev_fork);
    if (ix->ev_join) (void)hipEventDestroy(ix->ev_join);
    if (ix->ev_fork2) (void)hipEventDestroy(ix->ev_fork2);
    if (ix->ev_join2) (void)hipEventDestroy(ix->ev_join2);
    if (ix->stream) (void)hipStreamDestroy(ix->stream);
    delete ix;
}

// The side stream and its events (default priority); without them the query
// tables and the two-pass scans run on the search stream.
static void side_init(fbpq_index *ix)
{
    if (hipStreamCreateWithFlags(&ix->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ix->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ix->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ix->ev_fork2, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ix->ev_join2, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (ix->side) (void)hipStreamDestroy(ix->side);
        for (hipEvent_t e : {ix->ev_fork, ix->ev_join, ix->ev_fork2, ix->ev_join2})
            if (e) (void)hipEventDestroy(e);
        ix->side = nullptr;
        ix->ev_fork = ix->ev_join = ix->ev_fork2 = ix->ev_join2 = nullptr;
    }
}

int create_impl(const fbpq_index_desc *d, int device, fbpq_index **out)
{
    int rc = check_desc(d);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return fail(FBPQ_E_DEVICE, "device %d not available (%d devices)", device, ndev);
    }
    fbpq_index *ix = new fbpq_index();
    ix->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&ix->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete ix;
        return fail(FBPQ_E_DEVICE, "cannot initialise device %d", device);
    }
    {
        void *sp = nullptr;
        rc = scratch_addr(device, &sp);
        if (rc) {
            (void)hipStreamDestroy(ix->stream);
            delete ix;
            return rc;
        }
        side_init(ix);
        ix->arena.base = (unsigned char *)sp;
        ix->arena.cap = kScratchBytes;
    }
    scan_wide_prepare((int)d->M);  // kernel attributes read here, never inside a graph capture
    const int64_t T = d->T, h = d->D / 2, C = T * T, N = d->N, M = d->M;
    rc = upload(ix, &ix->C1, d->C1, sizeof(float) * T * h);
    if (!rc) rc = upload(ix, &ix->C2, d->C2, sizeof(float) * T * h);
    if (!rc) rc = upload(ix, &ix->R, d->R, sizeof(float) * M * FBPQ_KC * (d->D / M));
    if (!rc) rc = upload(ix, &ix->offsets, d->offsets, sizeof(int64_t) * (C + 1));
    if (!rc && d->QL) rc = upload(ix, &ix->QL, d->QL, sizeof(float) * T * FBPQ_KC * h);
    if (!rc && d->SL) rc = upload(ix, &ix->SL, d->SL, sizeof(float) * T * FBPQ_KC * h);
    if (!rc && d->Rot) rc = upload(ix, &ix->Rot, d->Rot, sizeof(float) * d->D * d->D);
    if (!rc) rc = upload(ix, &ix->ids, d->ids, sizeof(uint32_t) * N);
    if (!rc) {
        const size_t half = (size_t)N * (M / 2);
        if (hipMalloc(&ix->codesA, half ? half : 8) != hipSuccess ||
            hipMalloc(&ix->codesB, half ? half : 8) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(FBPQ_E_OOM, "device allocation of codes failed");
        } else {
            ix->base_bytes += 2 * half;
            // stage AoS codes through a bounded device buffer and split them on the GPU
            const int64_t step = std::max<int64_t>(1, ((int64_t)64 << 20) / M);
            void *stage = nullptr;
            rc = N ? ws_get(ix, W_SPLIT, (size_t)std::min(N, step) * M, &stage) : 0;
            for (int64_t s = 0; !rc && s < N; s += step) {
                const int64_t n = std::min(step, N - s);
                hipError_t e = hipMemcpy(stage, d->codes + s * M, (size_t)n * M, hipMemcpyHostToDevice);
                if (e == hipSuccess)
                    e = launch_split_codes((const uint8_t *)stage, n, (int)M, ix->codesA + s * (M / 2),
                                           ix->codesB + s * (M / 2), ix->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(ix->stream);
                if (e != hipSuccess) {
                    ix->poisoned = true;
                    rc = fail(FBPQ_E_DEVICE, "code upload failed: %s", hipGetErrorString(e));
                }
            }
            if (!rc && ix->ws[W_SPLIT].p) {
                (void)hipFree(ix->ws[W_SPLIT].p);
                ix->ws[W_SPLIT] = DevBuf{};
            }
        }
    }
    if (rc) {
        free_all(ix);
        return rc;
    }
    DevIndex &v = ix->dv;
    v.D = d->D;
    v.T = d->T;
    v.M = d->M;
    v.Kc = d->Kc;
    v.N = N;
    v.C1 = ix->C1;
    v.C2 = ix->C2;
    v.R = ix->R;
    v.offsets = ix->offsets;
    v.codesA = ix->codesA;
    v.codesB = ix->codesB;
    v.ids = ix->ids;
    v.QL = ix->QL;
    v.SL = ix->SL;
    v.Rot = ix->Rot;
    v.local = ix->QL ? 1 : 0;
    v.ecoef = 1.25f * (d->D / 2 + 8);
    *out = ix;
    return FBPQ_OK;
}

// ---- index file -------------------------------------------------------------
uint32_t crc_table[256];
bool crc_init = false;

uint32_t crc32_update(uint32_t crc, const unsigned char *p, size_t n)
{
    if (!crc_init) {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            crc_table[i] = c;
        }
        crc_init = true;
    }
    crc = ~crc;
    for (size_t i = 0; i < n; ++i) crc = crc_table[(crc ^ p[i]) & 255] ^ (crc >> 8);
    return ~crc;
}

#pragma pack(push, 1)
struct FileHdr {
    char magic[8];
    uint32_t version, D, T, M, Kc, nsect;
    uint64_t N;
    uint8_t reserved[24];
};
struct FileSec {
    uint32_t kind, crc;
    uint64_t offset, bytes, reserved;
};
#pragma pack(pop)
static_assert(sizeof(FileHdr) == 64, "header layout");
static_assert(sizeof(FileSec) == 32, "section layout");

// Sections 1-6 (C1, C2, R, offsets, codes, ids) are required; 7 and 8 (the
// local codebooks QL, SL, together) and 9 (the OPQ rotation) are optional.
constexpr int kSecReq = 6, kSecMax = 9;

struct FileData {
    FileHdr h;
    std::vector<float> C1, C2, R;
    std::vector<int64_t> offsets;
    std::vector<uint8_t> codes;
    std::vector<uint32_t> ids;
    std::vector<float> QL, SL, Rot;
    bool has[kSecMax] = {};
};

int read_file(const char *path, FileData *fd, bool keep)
{
    if (!path) return fail(FBPQ_E_INVALID, "null path");
    FILE *f = fopen(path, "rb");
    if (!f) return fail(FBPQ_E_IO, "cannot open %s", path);
    struct Closer {
        FILE *f;
        ~Closer() { fclose(f); }
    } closer{f};
    FileHdr &h = fd->h;
    if (fread(&h, sizeof h, 1, f) != 1) return fail(FBPQ_E_FORMAT, "%s: short header", path);
    if (memcmp(h.magic, "FBPQIDX1", 8) != 0) return fail(FBPQ_E_FORMAT, "%s: bad magic", path);
    if (h.version != 1) return fail(FBPQ_E_FORMAT, "%s: unsupported version %u", path, h.version);
    if (h.nsect < (uint32_t)kSecReq || h.nsect > (uint32_t)kSecMax)
        return fail(FBPQ_E_FORMAT, "%s: expected 6 to 9 sections", path);
    if (h.D == 0 || h.D % 2 || h.M == 0 || h.M % 2 || h.D % h.M || h.Kc != FBPQ_KC || h.T == 0 ||
        h.T > (1u << 20) || h.D > 4096 || h.N > 0xffffffffull)
        return fail(FBPQ_E_FORMAT, "%s: bad geometry", path);
    const int nsect = (int)h.nsect;
    FileSec sec[kSecMax];
    if (fread(sec, sizeof(FileSec), nsect, f) != (size_t)nsect)
        return fail(FBPQ_E_FORMAT, "%s: short section table", path);
    for (int s = 0; s < nsect; ++s) {
        if (sec[s].kind < 1 || sec[s].kind > (uint32_t)kSecMax) return fail(FBPQ_E_FORMAT, "%s: bad section kind", path);
        if (fd->has[sec[s].kind - 1]) return fail(FBPQ_E_FORMAT, "%s: section %u twice", path, sec[s].kind);
        fd->has[sec[s].kind - 1] = true;
    }
    for (int k = 0; k < kSecReq; ++k)
        if (!fd->has[k]) return fail(FBPQ_E_FORMAT, "%s: section %d missing", path, k + 1);
    if (fd->has[6] != fd->has[7]) return fail(FBPQ_E_FORMAT, "%s: local codebooks need both QL and SL", path);
    const uint64_t T = h.T, half = h.D / 2;
    const uint64_t want[kSecMax] = {4 * T * half, 4 * T * half, 4ull * h.M * h.Kc * (h.D / h.M),
                                    8 * (T * T + 1), h.N * h.M, 4 * h.N,
                                    4 * T * h.Kc * half, 4 * T * h.Kc * half, 4ull * h.D * h.D};
    void *dst[kSecMax] = {nullptr};
    if (keep) {
        fd->C1.resize(T * half);
        fd->C2.resize(T * half);
        fd->R.resize((size_t)h.M * h.Kc * (h.D / h.M));
        fd->offsets.resize(T * T + 1);
        fd->codes.resize(h.N * h.M);
        fd->ids.resize(h.N);
        if (fd->has[6]) fd->QL.resize(T * h.Kc * half);
        if (fd->has[7]) fd->SL.resize(T * h.Kc * half);
        if (fd->has[8]) fd->Rot.resize((size_t)h.D * h.D);
        void *d[kSecMax] = {fd->C1.data(), fd->C2.data(), fd->R.data(), fd->offsets.data(), fd->codes.data(),
                            fd->ids.data(), fd->QL.data(), fd->SL.data(), fd->Rot.data()};
        memcpy(dst, d, sizeof d);
    }
    std::vector<unsigned char> tmp;
    std::vector<int64_t> offs_check;
    for (int s = 0; s < nsect; ++s) {
        const FileSec &r = sec[s];
        const int k = (int)r.kind - 1;
        if (r.bytes != want[k]) return fail(FBPQ_E_FORMAT, "%s: section %d has %llu bytes, want %llu", path,
                                            k + 1, (unsigned long long)r.bytes, (unsigned long long)want[k]);
        if (fseeko(f, (off_t)r.offset, SEEK_SET) != 0) return fail(FBPQ_E_FORMAT, "%s: bad section offset", path);
        unsigned char *p;
        if (keep) {
            p = (unsigned char *)dst[k];
        } else if (k == 3) {
            offs_check.resize(T * T + 1);
            p = (unsigned char *)offs_check.data();
        } else {
            tmp.resize(std::min<uint64_t>(r.bytes, (uint64_t)1 << 24));
            p = nullptr;
        }
        uint32_t crc = 0;
        uint64_t left = r.bytes;
        uint64_t at = 0;
        while (left) {
            const size_t n = (size_t)std::min<uint64_t>(left, (uint64_t)1 << 24);
            unsigned char *q = p ? p + at : tmp.data();
            if (fread(q, 1, n, f) != n) return fail(FBPQ_E_FORMAT, "%s: truncated section %d", path, k + 1);
            crc = crc32_update(crc, q, n);
            left -= n;
            at += n;
        }
        if (crc != r.crc) return fail(FBPQ_E_FORMAT, "%s: CRC mismatch in section %d", path, k + 1);
    }
    const int64_t *o = keep ? fd->offsets.data() : offs_check.data();
    const int64_t C = (int64_t)T * T;
    if (o[0] != 0 || o[C] != (int64_t)h.N) return fail(FBPQ_E_FORMAT, "%s: offsets must span [0, N]", path);
    for (int64_t c = 0; c < C; ++c)
        if (o[c + 1] < o[c]) return fail(FBPQ_E_FORMAT, "%s: offsets decrease at cell %lld", path, (long long)c);
    return FBPQ_OK;
}

int check_handle(fbpq_index *ix)
{
    if (!ix) return fail(FBPQ_E_INVALID, "null index handle");
    if (ix->poisoned) return fail(FBPQ_E_DEVICE, "index handle poisoned by an earlier device error");
    if (hipSetDevice(ix->device) != hipSuccess) {
        (void)hipGetLastError();
        ix->poisoned = true;
        return fail(FBPQ_E_DEVICE, "cannot select device %d", ix->device);
    }
    return FBPQ_OK;
}

// ---- search pipeline ----------------------------------------------------------
struct DebugOut {
    // visit mode: traversal only, copy visited cells
    bool visit = false;
    int64_t cells_cap = 0;
    int64_t *cells = nullptr, *ncells = nullptr, *pos = nullptr, *npos = nullptr;
    int64_t pos_cap = 0;
    // dist mode: full pipeline, copy per-candidate distances
    bool dists = false;
    int64_t *dpos = nullptr;
    float *dd = nullptr;
    int64_t dcap = 0;
    int64_t *dn = nullptr;
};

#define TRY(x)                   \
    do {                         \
        int r_ = (x);            \
        if (r_) return r_;       \
    } while (0)

// First layer of a round: the sorted P-prefix of both half lists of every slot
// into lkey/lidx: the approximate key array of the round's slots, the
// wavefront select and, for the pairs it leaves over, the workgroup select.
int first_layer(fbpq_index *ix, const float *d_q, int64_t nslots, const int32_t *d_qlist, int32_t P,
                double *lkey, int32_t *lidx, hipStream_t st)
{
    const DevIndex &dv = ix->dv;
    void *pstat;
    TRY(ws_get(ix, W_PSTAT, sizeof(int32_t) * nslots * 2, &pstat));
    void *keys;
    TRY(ws_get(ix, W_KEYS, sizeof(float) * nslots * 2 * dv.T, &keys));
    const bool pwave = prefix_wave_ok(dv, P);
    void *kmin = nullptr;  // block minima: the wave select reads only the blocks that can hold survivors
    // (from T = 4096 on the minima save more reading than they cost the key kernel)
    const bool bmin = ix->block_min == 1 || (ix->block_min == 2 && dv.T >= 4096);
    if (pwave && bmin && prefix_blocks_ok(dv, P))
        TRY(ws_get(ix, W_KMIN, sizeof(float) * nslots * 2 * (size_t)((dv.T + 15) / 16), &kmin));
    HCK(ix, timed(ix, FBPQ_STAGE_HALF_KEYS, st, [&] { return launch_half_approx(dv, d_q, d_qlist, nslots, (float *)keys, (float *)kmin, st); }));
    if (pwave)
        HCK(ix, timed(ix, FBPQ_STAGE_PREFIX, st, [&] { return launch_prefix_wave(dv, d_q, (const float *)keys, (const float *)kmin, nslots, d_qlist, P, lkey, lidx, (int32_t *)pstat, ix->stats_dev, st); }));
    void *gsort = nullptr;  // long prefixes: the workgroup select sorts in HBM
    const size_t sort_bytes = prefix_sort_bytes(dv, P);
    if (sort_bytes) TRY(ws_get(ix, W_PSORT, sort_bytes * 2 * (size_t)nslots, &gsort));
    HCK(ix, timed(ix, pwave ? FBPQ_STAGE_PREFIX_FB : FBPQ_STAGE_PREFIX, st, [&] { return launch_prefix_block(dv, d_q, (const float *)keys, nslots, d_qlist, P, lkey, lidx, pwave ? (const int32_t *)pstat : nullptr, ix->stats_dev, (unsigned char *)gsort, st); }));
    return FBPQ_OK;
}

// One traversal round over nslots queries: launches every kernel of the
// round on st. With launch_only (graph capture) it stops there; otherwise it
// copies the debug outputs, waits for the stream and returns the number of
// queries that need another round.
int run_round(fbpq_index *ix, const float *d_q, int64_t nq, int64_t nslots, const int32_t *d_qlist,
              int32_t P, int64_t max_cells, int64_t lcap, const int64_t *d_L, const int32_t *d_k, int32_t k_max,
              int64_t *d_ids, float *d_d, hipStream_t st, int32_t *d_fail,
              const DebugOut *dbg, int64_t *fail_host_count, bool launch_only = false)
{
    DevIndex &dv = ix->dv;
    void *lkey, *lidx, *hdr, *w, *rowne, *rowcand, *colne, *coltot, *necs, *necnt, *nebeg, *necst, *cmcell,
        *cmpre;
    TRY(ws_get(ix, W_LKEY, sizeof(double) * nslots * 2 * P, &lkey));
    TRY(ws_get(ix, W_LIDX, sizeof(int32_t) * nslots * 2 * P, &lidx));
    TRY(ws_get(ix, W_HDR, sizeof(TravHdr) * nslots, &hdr));
    TRY(ws_get(ix, W_W, sizeof(int32_t) * nslots * P, &w));
    TRY(ws_get(ix, W_ROWNE, sizeof(int32_t) * nslots * (P + 1), &rowne));
    TRY(ws_get(ix, W_ROWCAND, sizeof(int32_t) * nslots * (P + 1), &rowcand));
    TRY(ws_get(ix, W_COLNE, sizeof(int32_t) * nslots * (P + 1), &colne));
    TRY(ws_get(ix, W_COLTOT, sizeof(int32_t) * nslots * P, &coltot));
    TRY(ws_get(ix, W_NECS, sizeof(int32_t) * nslots * max_cells, &necs));
    TRY(ws_get(ix, W_NECNT, sizeof(int32_t) * nslots * max_cells, &necnt));
    TRY(ws_get(ix, W_NEBEG, sizeof(int64_t) * nslots * max_cells, &nebeg));
    TRY(ws_get(ix, W_NECST, sizeof(float) * nslots * max_cells, &necst));
    TRY(ws_get(ix, W_CMCELL, sizeof(int32_t) * nslots * max_cells, &cmcell));
    TRY(ws_get(ix, W_CMPRE, sizeof(int32_t) * nslots * max_cells, &cmpre));
    void *neslot, *slotij;
    TRY(ws_get(ix, W_NESLOT, sizeof(int32_t) * nslots * max_cells, &neslot));
    TRY(ws_get(ix, W_SLOTIJ, sizeof(int32_t) * nslots * 2 * P, &slotij));
    void *dab = nullptr, *dtake = nullptr, *dbeg = nullptr, *dpos = nullptr, *ddd = nullptr;
    if (dbg && dbg->visit) {
        TRY(ws_get(ix, W_DBGAB, sizeof(int32_t) * 2 * nslots * max_cells, &dab));
        TRY(ws_get(ix, W_DBGTAKE, sizeof(int64_t) * nslots * max_cells, &dtake));
        TRY(ws_get(ix, W_DBGBEG, sizeof(int64_t) * nslots * max_cells, &dbeg));
    }
    if (dbg && dbg->dists) {
        TRY(ws_get(ix, W_DBGPOS, sizeof(int64_t) * nslots * dbg->dcap, &dpos));
        TRY(ws_get(ix, W_DBGD, sizeof(float) * nslots * dbg->dcap, &ddd));
    }
    HCK(ix, launch_fill_i32(d_fail, 0, 1, st));
    TRY(first_layer(ix, d_q, nslots, d_qlist, P, (double *)lkey, (int32_t *)lidx, st));
    // The query tables depend on the queries only: on the side stream they run
    // beside the traversal (forked after the first layer, which fills the chip), for every slot (the two-pass
    // scans, which do not read them, serve few queries), joined before the scans.
    const bool lq_need = !dv.local && !dv.od && !(dbg && dbg->visit);  // local and O(D) scans do not use LQ
    const bool lq_side = lq_need && ix->side && ix->ev_fork && ix->ev_join;
    void *lq = nullptr;
    if (lq_need) TRY(ws_get(ix, W_LQ, sizeof(float) * nslots * dv.M * FBPQ_KC, &lq));
    if (lq_side) {
        ItemArgs iq{};
        iq.ix = dv;
        iq.q = d_q;
        iq.qlist = d_qlist;
        iq.nslots = nslots;
        iq.hdr = nullptr;  // every slot
        iq.lq = (float *)lq;
        HCK(ix, hipEventRecord(ix->ev_fork, st));
        HCK(ix, hipStreamWaitEvent(ix->side, ix->ev_fork, 0));
        HCK(ix, timed(ix, FBPQ_STAGE_LQ, ix->side, [&] { return launch_items_prep(iq, ix->side); }));
        HCK(ix, hipEventRecord(ix->ev_join, ix->side));
    }
    TravArgs ta{};
    ta.ix = dv;
    ta.lkey = (const double *)lkey;
    ta.lidx = (const int32_t *)lidx;
    ta.P = P;
    ta.qlist = d_qlist;
    ta.L = d_L;
    ta.max_cells = max_cells;
    ta.hdr = (TravHdr *)hdr;
    ta.w = (int32_t *)w;
    ta.fail_count = d_fail;
    ta.fail_list = d_fail + 1;
    ta.dbg_ab = (int32_t *)dab;
    ta.dbg_take = (int64_t *)dtake;
    ta.dbg_beg = (int64_t *)dbeg;
    ta.stats = ix->stats_dev;
    // one cell at a time while the prefix fits its registers, then (for the
    // queries it leaves over, or all of them) the threshold-stepping kernel
    const bool pop = P <= kMaxPopPrefix && ix->pop_budget > 0;
    ta.pop_budget = pop ? ix->pop_budget : 0;
    ta.wide_all = pop ? 0 : 1;
    // prefixes longer than the LDS-resident kernels hold keep their per-rank state in HBM
    const bool big = P > kMaxFastPrefix;
    void *bigw = nullptr, *layscr = nullptr;
    if (big) {
        TRY(ws_get(ix, W_BIG, sizeof(int32_t) * (size_t)big_trav_ints(P) * nslots, &bigw));
        TRY(ws_get(ix, W_LAYSCR, layout_rank_bytes(P) * (size_t)nslots, &layscr));
        ta.big = (int32_t *)bigw;
    }
    if (pop) HCK(ix, timed(ix, FBPQ_STAGE_TRAVERSE, st, [&] { return launch_traverse(ta, nslots, st); }));
    if (big)
        HCK(ix, timed(ix, FBPQ_STAGE_TRAVERSE_WIDE, st, [&] { return launch_traverse_big(ta, nslots, st); }));
    else
        HCK(ix, timed(ix, FBPQ_STAGE_TRAVERSE_WIDE, st, [&] { return launch_traverse_wide(ta, nslots, st); }));
    if (!(dbg && dbg->visit)) {
        LayoutArgs la{};
        la.ix = dv;
        la.lkey = (const double *)lkey;
        la.lidx = (const int32_t *)lidx;
        la.P = P;
        la.hdr = (TravHdr *)hdr;
        la.w = (const int32_t *)w;
        la.max_cells = max_cells;
        la.row_ne = (int32_t *)rowne;
        la.row_cand = (int32_t *)rowcand;
        la.col_ne = (int32_t *)colne;
        la.col_tot = (int32_t *)coltot;
        la.ne_cs = (int32_t *)necs;
        la.ne_cnt = (int32_t *)necnt;
        la.ne_beg = (int64_t *)nebeg;
        la.ne_cst = (float *)necst;
        la.cm_cell = (int32_t *)cmcell;
        la.cm_pre = (int32_t *)cmpre;
        la.ne_slot = (int32_t *)neslot;
        la.slot_ij = (int32_t *)slotij;
        la.allow_items = ix->items ? 1 : 0;
        la.gscr = (unsigned char *)layscr;
        HCK(ix, timed(ix, FBPQ_STAGE_LAYOUT, st, [&] { return launch_layout(la, nslots, st); }));
        HCK(ix, timed(ix, FBPQ_STAGE_LAYOUT, st, [&] { return launch_layout_wide(la, nslots, st); }));
        // query tables and per-candidate distance rows: the cell scan and the
        // wide two-pass scan write the rows, the distance select reads them
        const int wcap = items_wcap(k_max);
        void *dist, *seldone;
        TRY(ws_get(ix, W_SELDONE, sizeof(int32_t) * nslots, &seldone));
        const int64_t dstride = (lcap + 63) & ~(int64_t)63;  // 256-byte aligned distance rows
        TRY(ws_get(ix, W_ITEMN, sizeof(float) * nslots * dstride, &dist));
        ItemArgs ia{};
        ia.ix = dv;
        ia.q = d_q;
        ia.qlist = d_qlist;
        ia.k = d_k;
        ia.k_max = k_max;
        ia.P = P;
        ia.nslots = nslots;
        ia.hdr = (const TravHdr *)hdr;
        ia.max_cells = max_cells;
        ia.ne_cs = (const int32_t *)necs;
        ia.ne_cnt = (const int32_t *)necnt;
        ia.ne_beg = (const int64_t *)nebeg;
        ia.ne_cst = (const float *)necst;
        ia.ne_slot = (const int32_t *)neslot;
        ia.slot_ij = (const int32_t *)slotij;
        ia.lq = (float *)lq;
        ia.dist = (float *)dist;
        ia.lcap = dstride;
        ia.wcap = wcap;
        ia.sel_done = (int32_t *)seldone;
        ia.stats = ix->stats_dev;
        ia.out_ids = d_ids;
        ia.out_d = d_d;
        ia.dbg_pos = (int64_t *)dpos;
        ia.dbg_d = (float *)ddd;
        ia.dbg_cap = dbg && dbg->dists ? dbg->dcap : 0;
        if (lq_side)
            HCK(ix, hipStreamWaitEvent(st, ix->ev_join, 0));
        else if (lq_need)
            HCK(ix, timed(ix, FBPQ_STAGE_LQ, st, [&] { return launch_items_prep(ia, st); }));
        ScanArgs sa{};
        sa.ix = dv;
        sa.q = d_q;
        sa.qlist = d_qlist;
        sa.k = d_k;
        sa.k_max = k_max;
        sa.lidx = (const int32_t *)lidx;
        sa.P = P;
        sa.hdr = (const TravHdr *)hdr;
        sa.max_cells = max_cells;
        sa.row_ne = (const int32_t *)rowne;
        sa.row_cand = (const int32_t *)rowcand;
        sa.col_ne = (const int32_t *)colne;
        sa.col_tot = (const int32_t *)coltot;
        sa.ne_cs = (const int32_t *)necs;
        sa.ne_cnt = (const int32_t *)necnt;
        sa.ne_beg = (const int64_t *)nebeg;
        sa.ne_cst = (const float *)necst;
        sa.cm_cell = (const int32_t *)cmcell;
        sa.cm_pre = (const int32_t *)cmpre;
        sa.ne_slot = (const int32_t *)neslot;
        sa.slot_ij = (const int32_t *)slotij;
        int chunk = ix->chunk;
        while (chunk > 256 && scan_lds_bytes(dv.D, dv.M, chunk, k_max, P) > kScanLdsLimit) chunk >>= 1;
        sa.chunk = chunk;
        sa.out_ids = d_ids;
        sa.out_d = d_d;
        sa.dbg_pos = (int64_t *)dpos;
        sa.dbg_d = (float *)ddd;
        sa.dbg_cap = dbg && dbg->dists ? dbg->dcap : 0;
        sa.stats = ix->stats_dev;
        sa.sel_done = (int32_t *)seldone;
        sa.lq = (const float *)lq;
        sa.dist = (float *)dist;
        sa.lcap = dstride;
        // the two-pass scans serve other slots than the cell scan, the wide scan
        // and the distance select: on the side stream they run beside them
        const bool s2_side = lq_side && ix->ev_fork2 && ix->ev_join2;
        if (s2_side) {
            HCK(ix, hipEventRecord(ix->ev_fork2, st));
            HCK(ix, hipStreamWaitEvent(ix->side, ix->ev_fork2, 0));
            HCK(ix, timed(ix, FBPQ_STAGE_SCAN2, ix->side, [&] { return launch_scan(sa, nslots, ix->side); }));
            HCK(ix, hipEventRecord(ix->ev_join2, ix->side));
        }
        if (ix->items && ix->persist) {
            PersistArgs pa{};
            void *pit, *pctl, *pqn, *pqd;
            TRY(ws_get(ix, W_PITEMS, sizeof(int32_t) * 3 * (size_t)persist_items_cap(nslots, dstride, ix->tile), &pit));
            TRY(ws_get(ix, W_PCTL, sizeof(int32_t) * 66, &pctl));
            TRY(ws_get(ix, W_PQNIT, sizeof(int32_t) * nslots, &pqn));
            TRY(ws_get(ix, W_PQDONE, sizeof(int32_t) * nslots, &pqd));
            pa.items = (int32_t *)pit;
            pa.ctl = (int32_t *)pctl;
            pa.qnit = (int32_t *)pqn;
            pa.qdone = (int32_t *)pqd;
            pa.tile = ix->tile;
            HCK(ix, timed(ix, FBPQ_STAGE_SCORE, st, [&] { return launch_items_persist(ia, pa, ix->pwaves, st); }));
        } else if (ix->items) {
            HCK(ix, timed(ix, FBPQ_STAGE_SCORE, st, [&] { return launch_items_scan(ia, st); }));
        }
        HCK(ix, timed(ix, FBPQ_STAGE_SCAN_WIDE, st, [&] { return launch_scan_wide(sa, nslots, st); }));
        HCK(ix, timed(ix, FBPQ_STAGE_SELECT, st, [&] { return launch_items_merge(ia, st); }));
        if (s2_side)
            HCK(ix, hipStreamWaitEvent(st, ix->ev_join2, 0));
        else
            HCK(ix, timed(ix, FBPQ_STAGE_SCAN2, st, [&] { return launch_scan(sa, nslots, st); }));
    }
    if (launch_only) return FBPQ_OK;
    // how many slots need another round
    // bytes [0, 64) of the pinned buffer hold the failure count; the L/k staging starts at 64
    void *pin;
    TRY(pinned_get(ix, 64, &pin));
    int32_t *hcount = (int32_t *)pin;
    HCK(ix, hipMemcpyAsync(hcount, d_fail, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (dbg && (dbg->visit || dbg->dists)) {
        // copy debug outputs of the successful slots to the caller
        std::vector<TravHdr> hh(nslots);
        std::vector<int32_t> ql(nslots);
        HCK(ix, hipMemcpyAsync(hh.data(), hdr, sizeof(TravHdr) * nslots, hipMemcpyDeviceToHost, st));
        if (d_qlist) HCK(ix, hipMemcpyAsync(ql.data(), d_qlist, sizeof(int32_t) * nslots, hipMemcpyDeviceToHost, st));
        HCK(ix, hipStreamSynchronize(st));
        if (!d_qlist)
            for (int64_t s = 0; s < nslots; ++s) ql[s] = (int32_t)s;
        if (dbg->visit) {
            std::vector<int32_t> ab((size_t)2 * nslots * max_cells);
            std::vector<int64_t> take((size_t)nslots * max_cells), beg((size_t)nslots * max_cells);
            std::vector<int32_t> li((size_t)nslots * 2 * P);
            std::vector<double> lk(P > kMaxFastPrefix ? (size_t)nslots * 2 * P : 0);
            if (!lk.empty()) HCK(ix, hipMemcpyAsync(lk.data(), lkey, lk.size() * 8, hipMemcpyDeviceToHost, st));
            HCK(ix, hipMemcpyAsync(ab.data(), dab, ab.size() * 4, hipMemcpyDeviceToHost, st));
            HCK(ix, hipMemcpyAsync(take.data(), dtake, take.size() * 8, hipMemcpyDeviceToHost, st));
            HCK(ix, hipMemcpyAsync(beg.data(), dbeg, beg.size() * 8, hipMemcpyDeviceToHost, st));
            HCK(ix, hipMemcpyAsync(li.data(), lidx, li.size() * 4, hipMemcpyDeviceToHost, st));
            HCK(ix, hipStreamSynchronize(st));
            for (int64_t s = 0; s < nslots; ++s) {
                if (hh[s].status != kStOk) continue;
                const int64_t q = ql[s];
                const int64_t nc = hh[s].ncells;
                if (nc > dbg->cells_cap || hh[s].ncand > dbg->pos_cap)
                    return fail(FBPQ_E_CAPACITY, "debug buffers too small for query %lld", (long long)q);
                // the long-prefix traversal lists its cells row-major: order them
                // by (key, a, b), the traversal order
                std::vector<int64_t> order((size_t)nc);
                for (int64_t c = 0; c < nc; ++c) order[c] = c;
                if (!lk.empty()) {
                    const double *k1 = lk.data() + (size_t)s * 2 * P, *k2 = k1 + P;
                    const int32_t *abs = ab.data() + (size_t)2 * s * max_cells;
                    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
                        const int32_t ax = abs[2 * x], bx = abs[2 * x + 1], ay = abs[2 * y], by = abs[2 * y + 1];
                        const double kx = k1[ax] + k2[bx], ky = k1[ay] + k2[by];
                        if (kx != ky) return kx < ky;
                        return ax != ay ? ax < ay : bx < by;
                    });
                }
                int64_t np = 0;
                for (int64_t ci = 0; ci < nc; ++ci) {
                    const int64_t c = ci;
                    const size_t o = (size_t)s * max_cells + order[ci];
                    const int32_t a = ab[2 * o], b = ab[2 * o + 1];
                    const int64_t cell = (int64_t)li[(size_t)s * 2 * P + a] * dv.T + li[(size_t)s * 2 * P + P + b];
                    dbg->cells[(q * dbg->cells_cap + c) * 2] = cell;
                    dbg->cells[(q * dbg->cells_cap + c) * 2 + 1] = take[o];
                    for (int64_t t = 0; t < take[o]; ++t) dbg->pos[q * dbg->pos_cap + np++] = beg[o] + t;
                }
                dbg->ncells[q] = nc;
                dbg->npos[q] = np;
            }
        }
        if (dbg->dists) {
            std::vector<int64_t> pp((size_t)nslots * dbg->dcap);
            std::vector<float> dd((size_t)nslots * dbg->dcap);
            HCK(ix, hipMemcpyAsync(pp.data(), dpos, pp.size() * 8, hipMemcpyDeviceToHost, st));
            HCK(ix, hipMemcpyAsync(dd.data(), ddd, dd.size() * 4, hipMemcpyDeviceToHost, st));
            HCK(ix, hipStreamSynchronize(st));
            for (int64_t s = 0; s < nslots; ++s) {
                if (hh[s].status != kStOk) continue;
                const int64_t q = ql[s];
                const int64_t n = hh[s].ncand;
                if (n > dbg->dcap) return fail(FBPQ_E_CAPACITY, "debug buffers too small");
                memcpy(dbg->dpos + q * dbg->dcap, pp.data() + s * dbg->dcap, n * 8);
                memcpy(dbg->dd + q * dbg->dcap, dd.data() + s * dbg->dcap, n * 4);
                dbg->dn[q] = n;
            }
        }
    }
    HCK(ix, hipStreamSynchronize(st));
    prof_collect(ix);
    *fail_host_count = hcount[0];
    return FBPQ_OK;
}

// An index with an OPQ rotation searches q' = Rot q: the rotated queries go
// to their own workspace slot (same address while nq stays, so a captured
// first round stays valid) and replace the caller's for the whole search.
int rotate_queries(fbpq_index *ix, const float **d_q, int64_t nq, hipStream_t st)
{
    if (!ix->dv.Rot) return FBPQ_OK;
    void *qr;
    TRY(ws_get(ix, W_QROT, sizeof(float) * (size_t)nq * ix->dv.D, &qr));
    const float *src = *d_q;
    HCK(ix, timed(ix, FBPQ_STAGE_ROTATE, st,
                  [&] { return launch_rotate(src, nq, ix->dv.D, ix->dv.Rot, (float *)qr, st); }));
    *d_q = (const float *)qr;
    return FBPQ_OK;
}

// What the retry rounds of a search need from its first round.
struct RoundCtx {
    const float *d_q;  // queries in the index's space
    int64_t nq;
    int32_t P;
    int64_t max_cells, lcap;
    const int64_t *dL;
    const int32_t *dk;
    int32_t *dfail;  // [0]: queries left for another round, then their ids
    int32_t k_max;
    int64_t *d_ids;
    float *d_d;
    hipStream_t st;
    const DebugOut *dbg;
};
int retry_rounds(fbpq_index *ix, RoundCtx &c, const int64_t *L, int64_t nfail);
int async_finish(fbpq_index *ix);

int search_impl(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                int32_t k_max, int64_t *d_ids, float *d_d, hipStream_t st, const DebugOut *dbg)
{
    if (ix && ix->async_open) TRY(async_finish(ix));
    TRY(check_handle(ix));
    struct CurStream {
        fbpq_index *ix;
        ~CurStream() { ix->cur = nullptr; }
    } cur_reset{ix};
    ix->cur = st;
    if (!ix->tables) return fail(FBPQ_E_STATE, "fbpq_build_tables has not been called");
    if (nq < 0) return fail(FBPQ_E_INVALID, "nq < 0");
    if (nq == 0) return FBPQ_OK;
    if (nq > 0x7fffffff) return fail(FBPQ_E_INVALID, "nq too large");
    if (!d_q || !L || !k) return fail(FBPQ_E_INVALID, "null pointer");
    if (k_max < 1 || k_max > FBPQ_K_MAX) return fail(FBPQ_E_INVALID, "k_max out of range");
    if (!(dbg && dbg->visit) && (!d_ids || !d_d)) return fail(FBPQ_E_INVALID, "null output");
    int64_t Lmax = 0;
    for (int64_t i = 0; i < nq; ++i) {
        if (L[i] < 1) return fail(FBPQ_E_INVALID, "L[%lld] < 1", (long long)i);
        if (k[i] < 1 || k[i] > k_max) return fail(FBPQ_E_INVALID, "k[%lld] out of [1, k_max]", (long long)i);
        Lmax = std::max(Lmax, L[i]);
    }
    if (std::min<int64_t>(Lmax, ix->dv.N) > 0x7fffffffLL)
        return fail(FBPQ_E_INVALID, "min(L, N) must stay below 2^31 candidates per query");
    void *dL, *dk, *dfail, *pin;
    TRY(ws_get(ix, W_L, sizeof(int64_t) * nq, &dL));
    TRY(ws_get(ix, W_K, sizeof(int32_t) * nq, &dk));
    TRY(ws_get(ix, W_FAIL, sizeof(int32_t) * (nq + 1), &dfail));
    TRY(pinned_get(ix, (sizeof(int64_t) + sizeof(int32_t)) * nq + 64, &pin));
    char *stage = (char *)pin + 64;
    memcpy(stage, L, sizeof(int64_t) * nq);
    memcpy(stage + sizeof(int64_t) * nq, k, sizeof(int32_t) * nq);
    HCK(ix, hipMemcpyAsync(dL, stage, sizeof(int64_t) * nq, hipMemcpyHostToDevice, st));
    HCK(ix, hipMemcpyAsync(dk, stage + sizeof(int64_t) * nq, sizeof(int32_t) * nq,
                           hipMemcpyHostToDevice, st));
    TRY(rotate_queries(ix, &d_q, nq, st));
    const int T = ix->dv.T;
    int32_t P = std::min<int32_t>(std::max<int32_t>(ix->prefix, 1), T);
    P = std::min<int32_t>(P, kMaxPrefix);
    int64_t max_cells = std::max<int64_t>(ix->max_cells, 64);
    const int64_t lcap = std::max<int64_t>(1, std::min(Lmax, ix->dv.N));
    if (ix->hint_first && !ix->graph) {
        // every query's budget class has needed a deeper traversal before (a
        // served batch holds one class): start there instead of retrying
        int32_t ph = INT32_MAX;
        int64_t ch = INT64_MAX;
        for (int64_t i = 0; i < nq && ph > 0; ++i) {
            const int b = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, std::min(L[i], ix->dv.N)));
            ph = std::min(ph, ix->p_hint[b]);
            ch = std::min(ch, ix->c_hint[b]);
        }
        if (ph > 0) {
            int32_t pmax = 0;
            int64_t cmax = 0;
            for (int64_t i = 0; i < nq; ++i) {
                const int b = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, std::min(L[i], ix->dv.N)));
                pmax = std::max(pmax, ix->p_hint[b]);
                cmax = std::max(cmax, ix->c_hint[b]);
            }
            const int32_t pc = std::min<int32_t>(std::min<int32_t>(T, kMaxPrefix), std::max<int32_t>(P, ix->prefix_cap));
            P = std::max(P, std::min(pmax, pc));
            int64_t c = max_cells;
            while (c < cmax && c < ((int64_t)1 << 26)) c *= 2;
            max_cells = c;
        }
        (void)ch;
    }
    int64_t nslots = nq;
    const int32_t *qlist = nullptr;
    int64_t nfail = 0;

    // first round: replay the captured graph when the launch sequence is the
    // same, else run it eagerly (and capture it for the next call)
    const bool use_graph = ix->graph && !dbg && !ix->profile && !ix->use_arena;
    fbpq_index::GraphKey key{d_q, nq, lcap, max_cells, ix->ws_gen, d_ids, d_d, k_max, P, ix->chunk, ix->pop_budget,
                             ix->items, ix->block_min, ix->persist, ix->tile, ix->pwaves, ix->stats_dev,
                             ix->dv.Cs1 != nullptr};
    if (use_graph && ix->gexec && ix->gkey == key) {
        HCK(ix, hipGraphLaunch(ix->gexec, st));
        ++ix->graph_replays;
        int32_t *hcount = (int32_t *)pin;  // bytes [0, 64) of the pinned buffer
        HCK(ix, hipMemcpyAsync(hcount, dfail, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HCK(ix, hipStreamSynchronize(st));
        nfail = hcount[0];
    } else {
        TRY(run_round(ix, d_q, nq, nslots, qlist, P, max_cells, lcap, (const int64_t *)dL, (const int32_t *)dk,
                      k_max, d_ids, d_d, st, (int32_t *)dfail, dbg, &nfail));
        if (use_graph) {
            // every workspace buffer of this shape exists now: capture the round
            hipStream_t cs = ix->stream;
            HCK(ix, hipStreamSynchronize(cs));
            const int64_t gen0 = ix->ws_gen;
            HCK(ix, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            const hipError_t e = hipSuccess;
            const int rc = run_round(ix, d_q, nq, nq, nullptr, P, max_cells, lcap, (const int64_t *)dL,
                                     (const int32_t *)dk, k_max, d_ids, d_d, cs, (int32_t *)dfail, nullptr, nullptr,
                                     true);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e != hipSuccess || rc != FBPQ_OK || e2 != hipSuccess || !g || ix->ws_gen != gen0) {
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                return rc != FBPQ_OK ? rc : fail(FBPQ_E_DEVICE, "graph capture of the search failed");
            }
            hipGraphExec_t ex = nullptr;
            const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HCK(ix, e3);
            if (ix->gexec) (void)hipGraphExecDestroy(ix->gexec);
            ix->gexec = ex;
            ix->gkey = key;
            ix->gkey.ws_gen = ix->ws_gen;
        }
    }
    RoundCtx c{d_q, nq, P, max_cells, lcap, (const int64_t *)dL, (const int32_t *)dk, (int32_t *)dfail, k_max,
               d_ids, d_d, st, dbg};
    return retry_rounds(ix, c, L, nfail);
}

// Retry rounds. A query whose traversal ran out of prefix ranks or cell
// capacity is searched again with 4x the ranks or 8x the cells; one that
// already had the most the traversal supports is a terminal failure: its
// result row is filled with (-2, NaN) and the others complete. The first
// round left nfail such queries (their list at c.dfail + 1); L holds the host
// copy of every query's budget.
int retry_rounds(fbpq_index *ix, RoundCtx &c, const int64_t *L, int64_t nfail)
{
    const float *d_q = c.d_q;
    const int64_t nq = c.nq;
    int32_t P = c.P;
    int64_t max_cells = c.max_cells;
    const int64_t lcap = c.lcap;
    const int32_t k_max = c.k_max;
    int64_t *d_ids = c.d_ids;
    float *d_d = c.d_d;
    hipStream_t st = c.st;
    const DebugOut *dbg = c.dbg;
    const void *dL = c.dL, *dk = c.dk;
    void *dfail = c.dfail;
    const int T = ix->dv.T;
    int64_t nslots = nq;
    const int32_t *qlist = nullptr;
    const int32_t Pcap = std::min<int32_t>(std::min<int32_t>(T, kMaxPrefix), std::max<int32_t>(P, ix->prefix_cap));
    const int64_t ccap = ((int64_t)1 << 31) / 32;
    std::vector<int32_t> cur;  // query of each slot of the last round (empty: slot = query)
    int64_t nterminal = 0;
    bool round_hint_set[64] = {false};  // hint buckets already written by this search
    auto record_hint = [&](int32_t q, int32_t Pq, int64_t cells) {
        const int b = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, std::min(L[q], ix->dv.N)));
        if (!round_hint_set[b]) {
            ix->p_hint[b] = Pq;
            ix->c_hint[b] = cells;
            round_hint_set[b] = true;
        } else {
            ix->p_hint[b] = std::max(ix->p_hint[b], Pq);
            ix->c_hint[b] = std::max(ix->c_hint[b], cells);
        }
    };
    // retry rounds take their buffers from the second workspace set, so that
    // they never move a buffer of the first round (and of its graph)
    struct WsBaseReset {
        fbpq_index *ix;
        ~WsBaseReset() { ix->ws_base = 0; }
    } ws_reset{ix};
    auto lbucket = [&](int32_t q) { return 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, std::min(L[q], ix->dv.N))); };
    for (int round = 1; nfail > 0; ++round) {
        ix->stat_retried += nfail;
        std::vector<TravHdr> hh(nslots);
        HCK(ix, hipMemcpyAsync(hh.data(), ws_ptr(ix, W_HDR), sizeof(TravHdr) * nslots,
                               hipMemcpyDeviceToHost, st));
        HCK(ix, hipStreamSynchronize(st));
        std::vector<int32_t> retry, terminal;
        bool grow_p = false, grow_c = false;
        int64_t need_cells = 0;  // cells a failed query is known to need (threshold kernel)
        for (int64_t sl = 0; sl < nslots; ++sl) {
            const int32_t q = cur.empty() ? (int32_t)sl : cur[sl];
            if (hh[sl].status == kStOk && !cur.empty()) record_hint(q, P, hh[sl].ncells);  // a retry round's success
            if (hh[sl].status != kStOk) need_cells = std::max(need_cells, hh[sl].ncells);
            if (hh[sl].status == kStNeedPrefix) {
                if (P >= Pcap) terminal.push_back(q);
                else {
                    retry.push_back(q);
                    grow_p = true;
                }
            } else if (hh[sl].status == kStNeedCells) {
                if (max_cells >= ccap) terminal.push_back(q);
                else {
                    retry.push_back(q);
                    grow_c = true;
                }
            }
        }
        if (!terminal.empty() && d_ids && d_d) {
            const std::vector<int64_t> rid((size_t)k_max, -2);
            const std::vector<float> rd((size_t)k_max, __builtin_nanf(""));
            for (int32_t q : terminal) {
                HCK(ix, hipMemcpyAsync(d_ids + (int64_t)q * k_max, rid.data(), sizeof(int64_t) * k_max,
                                       hipMemcpyHostToDevice, st));
                HCK(ix, hipMemcpyAsync(d_d + (int64_t)q * k_max, rd.data(), sizeof(float) * k_max,
                                       hipMemcpyHostToDevice, st));
            }
            HCK(ix, hipStreamSynchronize(st));
        }
        nterminal += (int64_t)terminal.size();
        if (grow_p) {
            int32_t Pn = std::min<int32_t>(Pcap, P * 4);
            for (size_t i = 0; i < retry.size(); ++i) {
                const int32_t hq = ix->p_hint[lbucket(retry[i])];
                if (hq > Pn) Pn = std::min<int32_t>(Pcap, hq);
            }
            P = Pn;
        }
        if (grow_c) max_cells = std::min<int64_t>(ccap, max_cells * 8);
        for (int32_t q : retry) need_cells = std::max(need_cells, ix->c_hint[lbucket(q)]);
        if (need_cells > max_cells) {
            // the next power of two: few distinct buffer sizes across batches
            int64_t c = max_cells;
            while (c < need_cells) c *= 2;
            max_cells = std::min<int64_t>(ccap, c);
        }
        if (retry.empty()) break;
        ix->ws_base = kWsSet;
        void *ql;
        TRY(ws_get(ix, W_QLIST, sizeof(int32_t) * retry.size(), &ql));
        HCK(ix, hipMemcpyAsync(ql, retry.data(), sizeof(int32_t) * retry.size(), hipMemcpyHostToDevice, st));
        qlist = (const int32_t *)ql;
        nslots = (int64_t)retry.size();
        cur.swap(retry);
        if (round > 64) return fail(FBPQ_E_CAPACITY, "traversal did not converge");
        nfail = 0;
        TRY(run_round(ix, d_q, nq, nslots, qlist, P, max_cells, lcap, (const int64_t *)dL, (const int32_t *)dk,
                      k_max, d_ids, d_d, st, (int32_t *)dfail, dbg, &nfail));
        if (nfail == 0) {
            // every query of this retry round succeeded at P
            std::vector<TravHdr> hl(nslots);
            HCK(ix, hipMemcpyAsync(hl.data(), ws_ptr(ix, W_HDR), sizeof(TravHdr) * nslots,
                                   hipMemcpyDeviceToHost, st));
            HCK(ix, hipStreamSynchronize(st));
            for (int64_t sl = 0; sl < nslots; ++sl) record_hint(cur[sl], P, hl[sl].ncells);
        }
    }
    if (nterminal)
        return fail(FBPQ_E_CAPACITY,
                    "%lld queries need more than %d ranks per half list or %lld cells (their rows are -2 / NaN)",
                    (long long)nterminal, Pcap, (long long)ccap);
    return FBPQ_OK;
}

// Completes the handle's open asynchronous search: waits for its first
// round, and runs its retry rounds on its stream if that round left queries.
int async_finish(fbpq_index *ix)
{
    if (!ix->async_open) return FBPQ_OK;
    ix->async_open = false;
    fbpq_index::AsyncState &a = ix->async;
    HCK(ix, hipEventSynchronize(ix->async_ev));
    const int64_t nfail = ix->async_count[0];
    if (nfail == 0) return FBPQ_OK;
    struct CurStream {
        fbpq_index *ix;
        ~CurStream() { ix->cur = nullptr; }
    } cur_reset{ix};
    ix->cur = a.st;
    void *dL = ws_ptr(ix, W_L), *dk = ws_ptr(ix, W_K), *dfail = ws_ptr(ix, W_FAIL);
    std::vector<int64_t> L((size_t)a.nq);
    HCK(ix, hipMemcpyAsync(L.data(), dL, sizeof(int64_t) * a.nq, hipMemcpyDeviceToHost, a.st));
    HCK(ix, hipStreamSynchronize(a.st));
    RoundCtx c{a.d_q, a.nq, a.P, a.max_cells, a.lcap, (const int64_t *)dL, (const int32_t *)dk, (int32_t *)dfail,
               a.k_max, a.d_ids, a.d_d, a.st, nullptr};
    return retry_rounds(ix, c, L.data(), nfail);
}

}  // namespace

namespace fbpq {

// A handle over the same index arrays with its own stream, workspace and
// pinned staging (one per concurrent batch of the serving layer). It copies
// the source handle's options. Freed with fbpq_free_index, which leaves the
// shared arrays alone; the source handle must outlive it.
int lane_create(fbpq_index *src, fbpq_index **out)
{
    TRY(check_handle(src));
    if (!src->tables) return fail(FBPQ_E_STATE, "fbpq_build_tables has not been called");
    fbpq_index *ix = new fbpq_index();
    ix->device = src->device;
    ix->shared = true;
    if (hipSetDevice(src->device) != hipSuccess ||
        hipStreamCreateWithFlags(&ix->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete ix;
        return fail(FBPQ_E_DEVICE, "cannot create a stream on device %d", src->device);
    }
    side_init(ix);
    ix->tables = true;
    ix->arena.base = src->arena.base;
    ix->arena.cap = src->arena.cap;
    ix->dv = src->dv;
    ix->C1 = src->C1;
    ix->C2 = src->C2;
    ix->R = src->R;
    ix->offsets = src->offsets;
    ix->codesA = src->codesA;
    ix->codesB = src->codesB;
    ix->ids = src->ids;
    ix->QL = src->QL;
    ix->SL = src->SL;
    ix->Rot = src->Rot;
    ix->CR1 = src->CR1;
    ix->CR2 = src->CR2;
    ix->nR = src->nR;
    ix->nC1 = src->nC1;
    ix->nC2 = src->nC2;
    ix->Cs1 = src->Cs1;
    ix->Cs2 = src->Cs2;
    ix->csc1 = src->csc1;
    ix->csc2 = src->csc2;
    ix->split_keys = src->split_keys;
    ix->prefix = src->prefix;
    ix->max_cells = src->max_cells;
    ix->chunk = src->chunk;
    ix->items = src->items;
    ix->block_min = src->block_min;
    ix->persist = src->persist;
    ix->hint_first = src->hint_first;
    ix->tile = src->tile;
    ix->pwaves = src->pwaves;
    ix->pop_budget = src->pop_budget;
    *out = ix;
    return FBPQ_OK;
}

int lane_device(const fbpq_index *ix) { return ix->device; }
int lane_dim(const fbpq_index *ix) { return ix->dv.D; }
int64_t lane_points(const fbpq_index *ix) { return ix->dv.N; }

int64_t search_ws_estimate(const fbpq_index *ix, int64_t L, int32_t k)
{
    const int64_t Leff = std::max<int64_t>(1, std::min(L, ix->dv.N));
    const int b = 63 - __builtin_clzll((unsigned long long)Leff);
    const int64_t T = ix->dv.T, M = ix->dv.M, D = ix->dv.D;
    const int64_t P = std::max<int64_t>(ix->prefix, ix->p_hint[b]);
    const int64_t cells = std::max<int64_t>(std::max<int64_t>(ix->max_cells, ix->c_hint[b]), 2 * Leff);
    // first round: keys, prefixes, per-rank arrays, cell lists, LQ, distance
    // row (a batch's stride is its largest min(L, N): at most 2 Leff within a
    // budget class), query, results
    const int64_t per_rank = 2 * P * 12 + 6 * (P + 1) * 4;
    const int64_t per_cell = 32;
    const int64_t once = 2 * T * 4 + M * kKc * 4 + D * 4 + (int64_t)k * 12 + 256;
    const int64_t round = per_rank + per_cell * cells;
    return once + 8 * Leff + 2 * round;  // the retry round has its own workspace set
}

}  // namespace fbpq

// ============================== C ABI ========================================
extern "C" {

const char *fbpq_last_error(void) { return g_err.c_str(); }

int fbpq_table_bytes(int64_t T, int64_t M, int64_t Kc, int64_t *table_bytes, int64_t *norm_bytes)
{
    if (T < 1 || M < 1 || Kc < 1 || !table_bytes || !norm_bytes) return fail(FBPQ_E_INVALID, "bad arguments");
    *table_bytes = T * M * Kc * (int64_t)sizeof(float);
    *norm_bytes = (2 * T + M * Kc) * (int64_t)sizeof(float);
    return FBPQ_OK;
}

int fbpq_index_create(const fbpq_index_desc *desc, int device, fbpq_index **out)
{
    if (!out) return fail(FBPQ_E_INVALID, "null output handle");
    *out = nullptr;
    return create_impl(desc, device, out);
}

int fbpq_index_file_check(const char *path, fbpq_info_t *info)
{
    FileData fd;
    const int rc = read_file(path, &fd, false);
    if (rc) return rc;
    if (info) {
        memset(info, 0, sizeof *info);
        info->D = (int32_t)fd.h.D;
        info->T = (int32_t)fd.h.T;
        info->M = (int32_t)fd.h.M;
        info->Kc = (int32_t)fd.h.Kc;
        info->N = (int64_t)fd.h.N;
        fbpq_table_bytes(info->T, info->M, info->Kc, &info->table_bytes, &info->norm_bytes);
        info->device = -1;
    }
    return FBPQ_OK;
}

int fbpq_load_index(const char *path, int device, fbpq_index **out)
{
    if (!out) return fail(FBPQ_E_INVALID, "null output handle");
    *out = nullptr;
    FileData fd;
    const int rc = read_file(path, &fd, true);
    if (rc) return rc;
    fbpq_index_desc d{};
    d.D = (int32_t)fd.h.D;
    d.T = (int32_t)fd.h.T;
    d.M = (int32_t)fd.h.M;
    d.Kc = (int32_t)fd.h.Kc;
    d.N = (int64_t)fd.h.N;
    d.C1 = fd.C1.data();
    d.C2 = fd.C2.data();
    d.R = fd.R.data();
    d.offsets = fd.offsets.data();
    d.codes = fd.codes.data();
    d.ids = fd.ids.data();
    d.QL = fd.has[6] ? fd.QL.data() : nullptr;
    d.SL = fd.has[7] ? fd.SL.data() : nullptr;
    d.Rot = fd.has[8] ? fd.Rot.data() : nullptr;
    return create_impl(&d, device, out);
}

// Approximate keys from the split FP16 half-centroids (when built and
// enabled) or from FP32 products, with the error coefficient that goes with
// them: 1.25 (h + 8) for FP32 sums of h products; 1.25 (2.5 h + 17) for the
// split form, whose sums run over 3 h exact products and drop terms below
// 3 2^-22 |q| |c|.
static void set_key_form(fbpq_index *ix)
{
    const int h = ix->dv.D / 2;
    const bool split = ix->split_keys && ix->Cs1 && ix->Cs2;
    ix->dv.Cs1 = split ? ix->Cs1 : nullptr;
    ix->dv.Cs2 = split ? ix->Cs2 : nullptr;
    ix->dv.csc1 = ix->csc1;
    ix->dv.csc2 = ix->csc2;
    ix->dv.ecoef = split ? 1.25f * (2.5f * h + 17.f) : 1.25f * (h + 8.f);
}

int fbpq_build_tables(fbpq_index *ix)
{
    TRY(check_handle(ix));
    if (ix->tables) return FBPQ_OK;
    const int64_t T = ix->dv.T, M = ix->dv.M;
    const size_t cr = sizeof(float) * T * (M / 2) * FBPQ_KC;
    const size_t nr = sizeof(float) * M * FBPQ_KC;
    if (hipMalloc(&ix->CR1, cr) != hipSuccess || hipMalloc(&ix->CR2, cr) != hipSuccess ||
        hipMalloc(&ix->nR, nr) != hipSuccess || hipMalloc(&ix->nC1, sizeof(float) * T) != hipSuccess ||
        hipMalloc(&ix->nC2, sizeof(float) * T) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FBPQ_E_OOM, "table allocation failed");
    }
    ix->table_bytes = 2 * cr + nr + 2 * sizeof(float) * T;
    HCK(ix, launch_tables(ix->dv, ix->CR1, ix->CR2, ix->nR, ix->nC1, ix->nC2, ix->stream));
    HCK(ix, hipStreamSynchronize(ix->stream));
    {
        std::vector<float> n1(T), n2(T);
        HCK(ix, hipMemcpy(n1.data(), ix->nC1, sizeof(float) * T, hipMemcpyDeviceToHost));
        HCK(ix, hipMemcpy(n2.data(), ix->nC2, sizeof(float) * T, hipMemcpyDeviceToHost));
        ix->dv.cmax1 = *std::max_element(n1.begin(), n1.end());
        ix->dv.cmax2 = *std::max_element(n2.begin(), n2.end());
    }
    if (ix->dv.D / 2 == 64) {
        // two-part FP16 half-centroids for the approximate keys, each half
        // scaled by a power of two to a largest magnitude below 2^14
        const int h = 64;
        const size_t sb = sizeof(_Float16) * T * 2 * h;
        if (hipMalloc(&ix->Cs1, sb) != hipSuccess || hipMalloc(&ix->Cs2, sb) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FBPQ_E_OOM, "table allocation failed");
        }
        std::vector<float> c((size_t)T * h);
        float *scs[2] = {&ix->csc1, &ix->csc2};
        const float *src[2] = {ix->C1, ix->C2};
        _Float16 *dst[2] = {ix->Cs1, ix->Cs2};
        for (int half = 0; half < 2; ++half) {
            HCK(ix, hipMemcpy(c.data(), src[half], sizeof(float) * c.size(), hipMemcpyDeviceToHost));
            float mx = 0.f;
            for (float x : c) mx = std::max(mx, std::fabs(x));
            int ex = 0;
            (void)std::frexp(mx, &ex);  // mx < 2^ex
            *scs[half] = std::ldexp(1.f, 14 - ex);
            HCK(ix, launch_split_centroids(src[half], T, h, *scs[half], dst[half], ix->stream));
        }
        HCK(ix, hipStreamSynchronize(ix->stream));
    }
    set_key_form(ix);
    ix->dv.CR1 = ix->CR1;
    ix->dv.CR2 = ix->CR2;
    ix->dv.nR = ix->nR;
    ix->dv.nC1 = ix->nC1;
    ix->dv.nC2 = ix->nC2;
    ix->tables = true;
    return FBPQ_OK;
}

int fbpq_search_device(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                       int32_t k_max, int64_t *d_ids, float *d_dists, void *hip_stream)
{
    return search_impl(ix, d_q, nq, L, k, k_max, d_ids, d_dists, (hipStream_t)hip_stream, nullptr);
}

int fbpq_search_device_async(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *d_L, const int32_t *d_k,
                             int64_t L_max, int32_t k_max, int64_t *d_ids, float *d_dists, int32_t *d_pending,
                             void *hip_stream)
{
    TRY(check_handle(ix));
    if (!ix->tables) return fail(FBPQ_E_STATE, "fbpq_build_tables has not been called");
    if (nq < 0 || nq > 0x7fffffff) return fail(FBPQ_E_INVALID, "nq out of range");
    if (L_max < 1) return fail(FBPQ_E_INVALID, "L_max < 1");
    if (k_max < 1 || k_max > FBPQ_K_MAX) return fail(FBPQ_E_INVALID, "k_max out of range");
    if (!d_pending || (nq > 0 && (!d_q || !d_L || !d_k || !d_ids || !d_dists)))
        return fail(FBPQ_E_INVALID, "null pointer");
    if (std::min<int64_t>(L_max, ix->dv.N) > 0x7fffffffLL)
        return fail(FBPQ_E_INVALID, "min(L_max, N) must stay below 2^31 candidates per query");
    TRY(async_finish(ix));  // the previous asynchronous search's retry rounds use the workspace
    hipStream_t st = (hipStream_t)hip_stream;
    struct CurStream {
        fbpq_index *ix;
        ~CurStream() { ix->cur = nullptr; }
    } cur_reset{ix};
    ix->cur = st;
    if (!ix->async_ev) {
        HCK(ix, hipEventCreateWithFlags(&ix->async_ev, hipEventDisableTiming));
        void *p = nullptr;
        if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FBPQ_E_OOM, "pinned host allocation failed");
        }
        ix->async_count = (int32_t *)p;
    }
    HCK(ix, launch_fill_i32(d_pending, 0, 2, st));
    if (nq == 0) return FBPQ_OK;
    void *dL, *dk, *dfail;
    TRY(ws_get(ix, W_L, sizeof(int64_t) * nq, &dL));
    TRY(ws_get(ix, W_K, sizeof(int32_t) * nq, &dk));
    TRY(ws_get(ix, W_FAIL, sizeof(int32_t) * (nq + 1), &dfail));
    HCK(ix, launch_sanitize(d_L, d_k, nq, L_max, k_max, (int64_t *)dL, (int32_t *)dk, d_pending + 1, st));
    TRY(rotate_queries(ix, &d_q, nq, st));
    const int T = ix->dv.T;
    const int32_t P = std::min<int32_t>(std::min<int32_t>(std::max<int32_t>(ix->prefix, 1), T), kMaxPrefix);
    const int64_t max_cells = std::max<int64_t>(ix->max_cells, 64);
    const int64_t lcap = std::max<int64_t>(1, std::min(L_max, ix->dv.N));
    const bool use_graph = ix->graph && !ix->profile;
    fbpq_index::GraphKey key{d_q, nq, lcap, max_cells, ix->ws_gen, d_ids, d_dists, k_max, P, ix->chunk,
                             ix->pop_budget, ix->items, ix->block_min, ix->persist, ix->tile, ix->pwaves,
                             ix->stats_dev};
    if (use_graph && ix->gexec && ix->gkey == key) {
        HCK(ix, hipGraphLaunch(ix->gexec, st));
        ++ix->graph_replays;
    } else {
        int64_t unused = 0;
        TRY(run_round(ix, d_q, nq, nq, nullptr, P, max_cells, lcap, (const int64_t *)dL, (const int32_t *)dk, k_max,
                      d_ids, d_dists, st, (int32_t *)dfail, nullptr, &unused, true));
    }
    HCK(ix, launch_copy_i32((const int32_t *)dfail, d_pending, st));
    HCK(ix, hipMemcpyAsync(ix->async_count, dfail, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HCK(ix, hipEventRecord(ix->async_ev, st));
    ix->async = fbpq_index::AsyncState{d_q, nq, P, max_cells, lcap, k_max, d_ids, d_dists, st};
    ix->async_open = true;
    return FBPQ_OK;
}

int fbpq_search_device_finish(fbpq_index *ix)
{
    TRY(check_handle(ix));
    return async_finish(ix);
}

int fbpq_search_device_noalloc(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                               int32_t k_max, int64_t *d_ids, float *d_dists, void *hip_stream)
{
    TRY(check_handle(ix));
    if (!ix->arena.base) return fail(FBPQ_E_STATE, "no scratch array on device %d", ix->device);
    struct ArenaOff {
        fbpq_index *ix;
        ~ArenaOff() { ix->use_arena = false; }
    } arena_off{ix};
    ix->arena.used = 0;
    for (int i = 0; i < 96; ++i) {
        ix->arena.slot[i] = nullptr;
        ix->arena.bytes[i] = 0;
    }
    ix->use_arena = true;
    return search_impl(ix, d_q, nq, L, k, k_max, d_ids, d_dists, (hipStream_t)hip_stream, nullptr);
}

static int host_search(fbpq_index *ix, const float *q, int64_t nq, const int64_t *L, const int32_t *k,
                       int32_t k_max, int64_t *ids, float *dists, const DebugOut *dbg)
{
    TRY(check_handle(ix));
    if (nq < 0) return fail(FBPQ_E_INVALID, "nq < 0");
    if (nq == 0) return ix->tables ? FBPQ_OK : fail(FBPQ_E_STATE, "fbpq_build_tables has not been called");
    if (!q) return fail(FBPQ_E_INVALID, "null queries");
    void *dq, *dids = nullptr, *dd = nullptr;
    TRY(ws_get(ix, W_Q, sizeof(float) * nq * ix->dv.D, &dq));
    const bool outputs = !(dbg && dbg->visit);
    if (outputs) {
        if (!ids || !dists) return fail(FBPQ_E_INVALID, "null output");
        TRY(ws_get(ix, W_IDS, sizeof(int64_t) * nq * k_max, &dids));
        TRY(ws_get(ix, W_D, sizeof(float) * nq * k_max, &dd));
    }
    HCK(ix, hipMemcpyAsync(dq, q, sizeof(float) * nq * ix->dv.D, hipMemcpyHostToDevice, ix->stream));
    // CAPACITY: some rows are marked (-2, NaN), the others are complete
    const int rc = search_impl(ix, (const float *)dq, nq, L, k, k_max, (int64_t *)dids, (float *)dd, ix->stream, dbg);
    if (rc && rc != FBPQ_E_CAPACITY) return rc;
    if (outputs) {
        HCK(ix, hipMemcpyAsync(ids, dids, sizeof(int64_t) * nq * k_max, hipMemcpyDeviceToHost, ix->stream));
        HCK(ix, hipMemcpyAsync(dists, dd, sizeof(float) * nq * k_max, hipMemcpyDeviceToHost, ix->stream));
        HCK(ix, hipStreamSynchronize(ix->stream));
    }
    return rc;
}

int fbpq_search_uneven(fbpq_index *ix, const float *q, int64_t nq, const int64_t *L, const int32_t *k,
                       int32_t k_max, int64_t *ids, float *dists)
{
    return host_search(ix, q, nq, L, k, k_max, ids, dists, nullptr);
}

int fbpq_search(fbpq_index *ix, const float *q, int64_t nq, int64_t L, int32_t k, int64_t *ids, float *dists)
{
    if (nq < 0) return fail(FBPQ_E_INVALID, "nq < 0");
    std::vector<int64_t> Ls((size_t)std::max<int64_t>(nq, 1), L);
    std::vector<int32_t> ks((size_t)std::max<int64_t>(nq, 1), k);
    if (k < 1 || k > FBPQ_K_MAX) return fail(FBPQ_E_INVALID, "k out of range");
    return host_search(ix, q, nq, Ls.data(), ks.data(), k, ids, dists, nullptr);
}

int fbpq_debug_visit(fbpq_index *ix, const float *q, int64_t nq, int64_t L, int64_t *cells, int64_t cells_cap,
                     int64_t *ncells, int64_t *pos, int64_t pos_cap, int64_t *npos)
{
    if (!cells || !ncells || !pos || !npos || cells_cap < 1 || pos_cap < 1)
        return fail(FBPQ_E_INVALID, "bad debug buffers");
    DebugOut dbg;
    dbg.visit = true;
    dbg.cells = cells;
    dbg.cells_cap = cells_cap;
    dbg.ncells = ncells;
    dbg.pos = pos;
    dbg.pos_cap = pos_cap;
    dbg.npos = npos;
    std::vector<int64_t> Ls((size_t)std::max<int64_t>(nq, 1), L);
    std::vector<int32_t> ks((size_t)std::max<int64_t>(nq, 1), 1);
    return host_search(ix, q, nq, Ls.data(), ks.data(), 1, nullptr, nullptr, &dbg);
}

int fbpq_debug_dists(fbpq_index *ix, const float *q, int64_t nq, int64_t L, int64_t *pos, float *dist,
                     int64_t cap, int64_t *n)
{
    if (!pos || !dist || !n || cap < 1) return fail(FBPQ_E_INVALID, "bad debug buffers");
    DebugOut dbg;
    dbg.dists = true;
    dbg.dpos = pos;
    dbg.dd = dist;
    dbg.dcap = cap;
    dbg.dn = n;
    std::vector<int64_t> Ls((size_t)std::max<int64_t>(nq, 1), L);
    std::vector<int32_t> ks((size_t)std::max<int64_t>(nq, 1), 1);
    std::vector<int64_t> ids((size_t)std::max<int64_t>(nq, 1));
    std::vector<float> dd((size_t)std::max<int64_t>(nq, 1));
    return host_search(ix, q, nq, Ls.data(), ks.data(), 1, ids.data(), dd.data(), &dbg);
}

int fbpq_debug_tables(fbpq_index *ix, float *CR1, float *CR2, float *nR, float *nC1, float *nC2)
{
    TRY(check_handle(ix));
    if (!ix->tables) return fail(FBPQ_E_STATE, "fbpq_build_tables has not been called");
    const int64_t T = ix->dv.T, M = ix->dv.M;
    const size_t cr = sizeof(float) * T * (M / 2) * FBPQ_KC;
    if (CR1) HCK(ix, hipMemcpy(CR1, ix->CR1, cr, hipMemcpyDeviceToHost));
    if (CR2) HCK(ix, hipMemcpy(CR2, ix->CR2, cr, hipMemcpyDeviceToHost));
    if (nR) HCK(ix, hipMemcpy(nR, ix->nR, sizeof(float) * M * FBPQ_KC, hipMemcpyDeviceToHost));
    if (nC1) HCK(ix, hipMemcpy(nC1, ix->nC1, sizeof(float) * T, hipMemcpyDeviceToHost));
    if (nC2) HCK(ix, hipMemcpy(nC2, ix->nC2, sizeof(float) * T, hipMemcpyDeviceToHost));
    return FBPQ_OK;
}

int fbpq_debug_rank(fbpq_index *ix, const float *q, int64_t nq, int32_t P, double *keys, int32_t *idx)
{
    TRY(check_handle(ix));
    if (nq < 0 || P < 1 || P > ix->dv.T || P > kMaxPrefix || !q || !keys || !idx)
        return fail(FBPQ_E_INVALID, "bad arguments");
    if (nq == 0) return FBPQ_OK;
    if (!ix->tables) return fail(FBPQ_E_STATE, "fbpq_build_tables has not been called");
    void *dq, *lkey, *lidx;
    TRY(ws_get(ix, W_Q, sizeof(float) * nq * ix->dv.D, &dq));
    TRY(ws_get(ix, W_LKEY, sizeof(double) * nq * 2 * P, &lkey));
    TRY(ws_get(ix, W_LIDX, sizeof(int32_t) * nq * 2 * P, &lidx));
    HCK(ix, hipMemcpyAsync(dq, q, sizeof(float) * nq * ix->dv.D, hipMemcpyHostToDevice, ix->stream));
    const float *qin = (const float *)dq;
    TRY(rotate_queries(ix, &qin, nq, ix->stream));
    TRY(first_layer(ix, qin, nq, nullptr, P, (double *)lkey, (int32_t *)lidx, ix->stream));
    HCK(ix, hipMemcpyAsync(keys, lkey, sizeof(double) * nq * 2 * P, hipMemcpyDeviceToHost, ix->stream));
    HCK(ix, hipMemcpyAsync(idx, lidx, sizeof(int32_t) * nq * 2 * P, hipMemcpyDeviceToHost, ix->stream));
    HCK(ix, hipStreamSynchronize(ix->stream));
    return FBPQ_OK;
}

int fbpq_info(const fbpq_index *ix, fbpq_info_t *out)
{
    if (!ix || !out) return fail(FBPQ_E_INVALID, "null argument");
    if (ix->poisoned) return fail(FBPQ_E_DEVICE, "index handle poisoned by an earlier device error");
    memset(out, 0, sizeof *out);
    out->D = ix->dv.D;
    out->T = ix->dv.T;
    out->M = ix->dv.M;
    out->Kc = ix->dv.Kc;
    out->N = ix->dv.N;
    fbpq_table_bytes(out->T, out->M, out->Kc, &out->table_bytes, &out->norm_bytes);
    size_t ws = 0;
    for (const auto &b : ix->ws) ws += b.cap;
    out->device_bytes = (int64_t)(ix->base_bytes + ix->table_bytes + ws);
    out->tables_ready = ix->tables ? 1 : 0;
    out->device = ix->device;
    return FBPQ_OK;
}

int fbpq_set_option(fbpq_index *ix, const char *key, int64_t value)
{
    if (!ix || !key) return fail(FBPQ_E_INVALID, "null argument");
    if (ix->poisoned) return fail(FBPQ_E_DEVICE, "index handle poisoned by an earlier device error");
    if (!strcmp(key, "prefix")) {
        if (value < 1 || value > kMaxPrefix) return fail(FBPQ_E_INVALID, "prefix out of [1, %d]", kMaxPrefix);
        ix->prefix = (int32_t)value;
    } else if (!strcmp(key, "prefix_cap")) {
        if (value < 1 || value > kMaxPrefix) return fail(FBPQ_E_INVALID, "prefix_cap out of [1, %d]", kMaxPrefix);
        ix->prefix_cap = (int32_t)value;
    } else if (!strcmp(key, "max_cells")) {
        if (value < 64 || value > ((int64_t)1 << 26)) return fail(FBPQ_E_INVALID, "max_cells out of range");
        ix->max_cells = value;
    } else if (!strcmp(key, "hint_first")) {
        ix->hint_first = value != 0;
    } else if (!strcmp(key, "persist")) {
        ix->persist = value != 0;
    } else if (!strcmp(key, "tile")) {
        if (value < 64 || value > ((int64_t)1 << 30)) return fail(FBPQ_E_INVALID, "tile out of [64, 2^30]");
        ix->tile = (int32_t)value;
    } else if (!strcmp(key, "pwaves")) {
        if (value != 2 && value != 4 && value != 8) return fail(FBPQ_E_INVALID, "pwaves must be 2, 4 or 8");
        ix->pwaves = (int32_t)value;
    } else if (!strcmp(key, "block_min")) {
        if (value < 0 || value > 2) return fail(FBPQ_E_INVALID, "block_min must be 0, 1 or 2");
        ix->block_min = (int32_t)value;
    } else if (!strcmp(key, "items")) {
        ix->items = value != 0;
    } else if (!strcmp(key, "profile")) {
        ix->profile = value != 0;
    } else if (!strcmp(key, "profile_mask")) {
        ix->prof_mask = value;
    } else if (!strcmp(key, "inject_device_error")) {
        if (value < 0) return fail(FBPQ_E_INVALID, "inject_device_error < 0");
        ix->inject_after = value;
    } else if (!strcmp(key, "split_keys")) {
        ix->split_keys = value != 0;
        set_key_form(ix);
    } else if (!strcmp(key, "graph")) {
        ix->graph = value != 0;
        if (!ix->graph && ix->gexec) {
            HCK(ix, hipDeviceSynchronize());
            (void)hipGraphExecDestroy(ix->gexec);
            ix->gexec = nullptr;
        }
    } else if (!strcmp(key, "stats")) {
        if (value) {
            HCK(ix, hipSetDevice(ix->device));
            if (!ix->stats_dev) {
                void *p = nullptr;
                HCK(ix, hipMalloc(&p, sizeof(unsigned long long) * kNumStatSlots));
                ix->stats_dev = (unsigned long long *)p;
            }
            HCK(ix, hipMemset(ix->stats_dev, 0, sizeof(unsigned long long) * kNumStatSlots));
            ix->stat_retried = 0;
            ix->graph_replays = 0;
        } else if (ix->stats_dev) {
            HCK(ix, hipDeviceSynchronize());
            (void)hipFree(ix->stats_dev);
            ix->stats_dev = nullptr;
        }
    } else if (!strcmp(key, "adc_od")) {
        // score every candidate by explicit reconstruction (the Multi-D-ADC baseline)
        ix->dv.od = value != 0 ? 1 : 0;
        if (ix->gexec) {
            HCK(ix, hipDeviceSynchronize());
            (void)hipGraphExecDestroy(ix->gexec);
            ix->gexec = nullptr;
        }
    } else if (!strcmp(key, "pop_budget")) {
        if (value < 0 || value > ((int64_t)1 << 26)) return fail(FBPQ_E_INVALID, "pop_budget out of range");
        ix->pop_budget = (int32_t)value;
    } else if (!strcmp(key, "chunk")) {
        if (value < 256 || value > (1 << 16)) return fail(FBPQ_E_INVALID, "chunk out of range");
        ix->chunk = (int32_t)value;
    } else {
        return fail(FBPQ_E_INVALID, "unknown option %s", key);
    }
    return FBPQ_OK;
}

int fbpq_profile_read(fbpq_index *ix, int32_t stage, int32_t reset, double *ms, int64_t *launches)
{
    if (!ix || stage < 0 || stage >= FBPQ_NUM_STAGES || !ms || !launches)
        return fail(FBPQ_E_INVALID, "bad arguments");
    if (ix->poisoned) return fail(FBPQ_E_DEVICE, "index handle poisoned by an earlier device error");
    *ms = ix->prof_ms[stage];
    *launches = ix->prof_n[stage];
    if (reset) {
        ix->prof_ms[stage] = 0;
        ix->prof_n[stage] = 0;
    }
    return FBPQ_OK;
}

// Times one setting: a warm search, then `reps` timed with HIP events; the median.
static int tune_time(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k, int32_t k_max,
                     int64_t *d_ids, float *d_dists, hipStream_t st, int32_t reps, hipEvent_t e0, hipEvent_t e1,
                     double *ms_out)
{
    int rc = search_impl(ix, d_q, nq, L, k, k_max, d_ids, d_dists, st, nullptr);  // warm: workspace, retries
    if (rc) return rc;
    std::vector<float> t(reps);
    for (int r = 0; r < reps; ++r) {
        if (hipEventRecord(e0, st) != hipSuccess) return fail(FBPQ_E_DEVICE, "event record failed");
        rc = search_impl(ix, d_q, nq, L, k, k_max, d_ids, d_dists, st, nullptr);
        if (rc) return rc;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
            return fail(FBPQ_E_DEVICE, "event timing failed");
    }
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return FBPQ_OK;
}

struct TuneChoice {
    int32_t prefix, items, persist, tile, pwaves;
    double ms;
};

// A candidate starts from no learned budget-class hints: hints left by an
// earlier candidate's retries would start every later one at that depth.
static void tune_apply(fbpq_index *ix, const TuneChoice &c)
{
    std::fill(std::begin(ix->p_hint), std::end(ix->p_hint), 0);
    std::fill(std::begin(ix->c_hint), std::end(ix->c_hint), 0);
    ix->prefix = c.prefix;
    ix->items = c.items != 0;
    ix->persist = c.persist != 0;
    ix->tile = c.tile;
    ix->pwaves = c.pwaves;
}

// Coordinate search: first the sorted-prefix length and the scan form, then
// (cell scan only) the persistent scan's tile and wavefronts per workgroup
// against the per-query launch.
static int tune_run(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k, int32_t k_max,
                    int64_t *d_ids, float *d_dists, hipStream_t st, int32_t reps, TuneChoice *best)
{
    const int32_t T = ix->dv.T;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HCK(ix, hipEventCreate(&e0));
    HCK(ix, hipEventCreate(&e1));
    int rc = FBPQ_OK;
    TuneChoice b{std::min<int32_t>(T, kMaxPrefix), 1, 0, ix->tile, ix->pwaves, -1.0};
    auto consider = [&](const TuneChoice &c) {
        if (rc) return;
        tune_apply(ix, c);
        double ms = 0.0;
        rc = tune_time(ix, d_q, nq, L, k, k_max, d_ids, d_dists, st, reps, e0, e1, &ms);
        if (!rc && (b.ms < 0 || ms < b.ms)) {
            b = c;
            b.ms = ms;
        }
    };
    // Stage 1 times every (prefix, scan form) twice, round robin, and keeps
    // each one's faster median: the first candidates of a single pass would
    // run while the clocks still rise after the caller's own work.
    std::vector<TuneChoice> c1;
    for (int32_t p : {16, 32, 64, 128, 256, 512})  // short prefixes retry the queries they do not cover
        if (p <= std::min<int32_t>(T, kMaxPrefix)) {
            c1.push_back({p, 1, 0, ix->tile, ix->pwaves, -1.0});
            c1.push_back({p, 0, 0, ix->tile, ix->pwaves, -1.0});
        }
    for (int pass = 0; pass < 2 && !rc; ++pass)
        for (TuneChoice &c : c1) {
            if (rc) break;
            tune_apply(ix, c);
            double ms = 0.0;
            rc = tune_time(ix, d_q, nq, L, k, k_max, d_ids, d_dists, st, reps, e0, e1, &ms);
            if (!rc && (c.ms < 0 || ms < c.ms)) c.ms = ms;
        }
    for (const TuneChoice &c : c1)
        if (!rc && (b.ms < 0 || c.ms < b.ms)) b = c;
    if (c1.empty()) consider(b);
    if (!rc && b.items) {
        const int mh = ix->dv.M / 2;
        for (int32_t tile : {2048, 8192, 32768, 1 << 30})
            for (int32_t w : {2, 4, 8}) {
                if ((w == 2 && mh > 4) || (w == 8 && mh < 2)) continue;  // the shapes the kernel is built for
                consider({b.prefix, 1, 1, tile, w, 0.0});
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = b;
    return FBPQ_OK;
}

static void tune_out(const TuneChoice &c, int64_t *chosen)
{
    chosen[0] = c.prefix;
    chosen[1] = c.items;
    chosen[2] = (int64_t)(c.ms * 1000.0);  // microseconds per search of the batch
    chosen[3] = c.persist;
    chosen[4] = c.tile;
    chosen[5] = c.pwaves;
}

int fbpq_autotune(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                  int32_t k_max, int64_t *d_ids, float *d_dists, void *hip_stream, int32_t reps, int64_t *chosen)
{
    TRY(check_handle(ix));
    if (reps < 1 || reps > 100 || !chosen) return fail(FBPQ_E_INVALID, "bad autotune arguments");
    const bool prof0 = ix->profile, graph0 = ix->graph;
    const TuneChoice keep{ix->prefix, ix->items ? 1 : 0, ix->persist ? 1 : 0, ix->tile, ix->pwaves, 0.0};
    ix->profile = false;
    ix->graph = false;
    TuneChoice best{};
    const int rc = tune_run(ix, d_q, nq, L, k, k_max, d_ids, d_dists, (hipStream_t)hip_stream, reps, &best);
    ix->profile = prof0;
    ix->graph = graph0;
    if (rc) {
        tune_apply(ix, keep);
        return rc;
    }
    tune_apply(ix, best);
    tune_out(best, chosen);
    return FBPQ_OK;
}

// The tuning cache key: geometry, batch size class, budget classes (log2 of
// the mean min(L, N) and of k_max) and the device (architecture and compute
// unit count).
static int tune_key(fbpq_index *ix, int64_t nq, const int64_t *L, int32_t k_max, std::string *key)
{
    double sum = 0.0;
    for (int64_t i = 0; i < nq; ++i) sum += (double)std::min(L[i], ix->dv.N);
    const int64_t mean = nq ? (int64_t)(sum / (double)nq) : 1;
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, ix->device) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FBPQ_E_DEVICE, "cannot read the device properties");
    }
    char buf[512];
    snprintf(buf, sizeof buf, "D=%d T=%d M=%d N=%lld nq2=%d L2=%d k2=%d local=%d dev=%s/%d", ix->dv.D, ix->dv.T,
             ix->dv.M, (long long)ix->dv.N, 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, nq)),
             63 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, mean)),
             31 - __builtin_clz((unsigned)std::max(1, k_max)), ix->dv.local, prop.gcnArchName,
             prop.multiProcessorCount);
    *key = buf;
    return FBPQ_OK;
}

static std::mutex g_tune_mu;

// One JSON object per line: {"key": "...", "prefix": P, "items": I,
// "persist": S, "tile": W, "pwaves": V, "us": U}. The last record of a key wins.
static bool tune_lookup(const char *path, const std::string &key, TuneChoice *c)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    const std::string want = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, want.c_str())) continue;
        const char *p = strstr(line, "\"prefix\":");
        TuneChoice t{};
        long long us = 0;
        if (p && sscanf(p, "\"prefix\": %d, \"items\": %d, \"persist\": %d, \"tile\": %d, \"pwaves\": %d, \"us\": %lld",
                        &t.prefix, &t.items, &t.persist, &t.tile, &t.pwaves, &us) == 6) {
            t.ms = (double)us / 1000.0;
            *c = t;
            found = true;
        }
    }
    fclose(f);
    return found;
}

int fbpq_autotune_cached(fbpq_index *ix, const float *d_q, int64_t nq, const int64_t *L, const int32_t *k,
                         int32_t k_max, int64_t *d_ids, float *d_dists, void *hip_stream, int32_t reps,
                         const char *cache_path, int64_t *chosen, int32_t *from_cache)
{
    TRY(check_handle(ix));
    if (!cache_path || !from_cache || !chosen || !L || nq < 1) return fail(FBPQ_E_INVALID, "bad autotune arguments");
    std::string key;
    TRY(tune_key(ix, nq, L, k_max, &key));
    TuneChoice c{};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (tune_lookup(cache_path, key, &c)) {
            const bool ok = c.prefix >= 1 && c.prefix <= kMaxPrefix && c.tile >= 64 &&
                            (c.pwaves == 2 || c.pwaves == 4 || c.pwaves == 8);
            if (ok) {
                tune_apply(ix, c);
                tune_out(c, chosen);
                *from_cache = 1;
                return FBPQ_OK;
            }
        }
    }
    TRY(fbpq_autotune(ix, d_q, nq, L, k, k_max, d_ids, d_dists, hip_stream, reps, chosen));
    *from_cache = 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = fopen(cache_path, "a");
    if (!f) return fail(FBPQ_E_IO, "cannot append to %s", cache_path);
    fprintf(f, "{\"key\": \"%s\", \"prefix\": %lld, \"items\": %lld, \"persist\": %lld, \"tile\": %lld, \"pwaves\": %lld, "
               "\"us\": %lld}\n",
            key.c_str(), (long long)chosen[0], (long long)chosen[1], (long long)chosen[3], (long long)chosen[4],
            (long long)chosen[5], (long long)chosen[2]);
    fclose(f);
    return FBPQ_OK;
}

int fbpq_stats_read(fbpq_index *ix, int64_t *out, int32_t n, int32_t reset)
{
    TRY(check_handle(ix));
    if (!out || n < 0) return fail(FBPQ_E_INVALID, "bad arguments");
    if (!ix->stats_dev) return fail(FBPQ_E_STATE, "path counters are off (option \"stats\")");
    HCK(ix, hipSetDevice(ix->device));
    unsigned long long h[kNumStatSlots];
    HCK(ix, hipDeviceSynchronize());
    HCK(ix, hipMemcpy(h, ix->stats_dev, sizeof(h), hipMemcpyDeviceToHost));
    h[FBPQ_STAT_RETRIED] = (unsigned long long)ix->stat_retried;
    h[FBPQ_STAT_GRAPH_REPLAYS] = (unsigned long long)ix->graph_replays;
    for (int i = 0; i < n && i < FBPQ_NUM_STATS; ++i) out[i] = (int64_t)h[i];
    if (reset) {
        HCK(ix, hipMemset(ix->stats_dev, 0, sizeof(h)));
        ix->stat_retried = 0;
        ix->graph_replays = 0;
    }
    return FBPQ_OK;
}

void fbpq_free_index(fbpq_index *ix) { free_all(ix); }

}  // extern "C"
