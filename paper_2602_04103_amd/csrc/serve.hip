// Native serving loop for FM-index count requests: continuous batching against a device-resident
// QuadFm index, the host-side core behind the serving row.
//
// Requests arrive over time (their arrival times are given), each holding a contiguous block of
// patterns.  Whenever a slot (a stream with its own work-queue head) is free, every request that has
// arrived is admitted FIFO as one batch, as large as the pattern cap and the device arena allow; an
// optional live free-memory check can also hold admission back, and the arena can grow from the
// device's free memory (chunks of at least the budget, kept above a headroom).  A batch moves its
// pattern bytes (one per base, or 2-bit packed words) and offsets into the arena, rebasing the
// offsets, runs the persistent count kernel on the slot's stream, moves the counts back and records
// an event.  The moves are kernels that read and write the caller's pinned host memory when the
// batch is small (no copy call, whose rare multi-millisecond pauses would hold up the whole loop)
// and DMA copies otherwise.  Up to `slots` batches are in flight at once, so batches that arrive
// while others run overlap on the device.  A request finishes when the host sees its batch's event
// complete.
//
// The policy (FIFO batches, first-fit arena of 256-byte aligned blocks, batch byte budget) is the
// same as the scheduler the Python tests exercise with a CPU stand-in.
#include <algorithm>
#include <chrono>
#include <new>
#include <utility>
#include <vector>

#include "common.hpp"

using namespace qr;

namespace {

constexpr uint64_t ALIGN = 256;

uint64_t pad(uint64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over a list of chunks, each [0, size): per chunk sorted, disjoint, coalesced
// free ranges; a block never spans two chunks.
struct Arena {
    std::vector<uint64_t> size;
    std::vector<std::vector<std::pair<uint64_t, uint64_t>>> free_;

    void add(uint64_t s) {
        size.push_back(s);
        free_.push_back({{0, s}});
    }
    uint64_t largest() const { return size.empty() ? 0 : *std::max_element(size.begin(), size.end()); }
    bool alloc(uint64_t nbytes, uint32_t &chunk, uint64_t &at) {
        for (size_t c = 0; c < free_.size(); ++c) {
            auto &fr = free_[c];
            for (size_t k = 0; k < fr.size(); ++k) {
                const uint64_t a = fr[k].first, b = fr[k].second;
                const uint64_t s = (a + ALIGN - 1) / ALIGN * ALIGN;
                if (s + nbytes <= b) {
                    std::vector<std::pair<uint64_t, uint64_t>> pieces;
                    if (s > a) pieces.push_back({a, s});
                    if (s + nbytes < b) pieces.push_back({s + nbytes, b});
                    fr.erase(fr.begin() + k);
                    fr.insert(fr.begin() + k, pieces.begin(), pieces.end());
                    chunk = (uint32_t)c;
                    at = s;
                    return true;
                }
            }
        }
        return false;
    }
    void release(uint32_t chunk, uint64_t start, uint64_t nbytes) {
        auto &fr = free_[chunk];
        const std::pair<uint64_t, uint64_t> blk{start, start + nbytes};
        fr.insert(std::lower_bound(fr.begin(), fr.end(), blk), blk);
        std::vector<std::pair<uint64_t, uint64_t>> merged;
        for (const auto &r : fr) {
            if (!merged.empty() && merged.back().second >= r.first)
                merged.back().second = std::max(merged.back().second, r.second);
            else
                merged.push_back(r);
        }
        fr.swap(merged);
    }
};

// off[i] -= base for i < n: the batch's offsets, copied as they are, made relative to its first byte
// (packed patterns: to the first base of its first word)
__global__ void rebase_offsets(uint64_t *__restrict__ off, uint64_t n, uint64_t base) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) off[i] -= base;
}

// Direct batches (pinned, device-mapped host buffers): the GPU reads the batch's pattern bytes and
// offsets from host memory into the arena, rebasing the offsets, and writes the counts back, so a
// batch is launches only (no DMA copies).  src and dst of the pattern copy are both 8-byte aligned
// when src is (dst is an arena block); the copy then moves u64 words and the tail bytes.
__global__ void stage_in(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src, uint64_t nbytes,
                         uint64_t *__restrict__ doff, const uint64_t *__restrict__ soff, uint64_t noff, uint64_t base) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t head = 0;
    if (((uintptr_t)src & 7) == 0) {
        head = nbytes / 8 * 8;
        const uint64_t *s8 = reinterpret_cast<const uint64_t *>(src);
        uint64_t *d8 = reinterpret_cast<uint64_t *>(dst);
        for (uint64_t i = t; i < nbytes / 8; i += stride) d8[i] = s8[i];
    }
    for (uint64_t i = head + t; i < nbytes; i += stride) dst[i] = src[i];
    for (uint64_t i = t; i < noff; i += stride) doff[i] = soff[i] - base;
}

__global__ void stage_out(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src, uint64_t n) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = t; i < n; i += stride) dst[i] = src[i];
}

uint32_t stage_blocks(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 1024)); }

// Device address of the host range [p, p + len) if the GPU can access it directly: pinned host
// memory mapped for the device (hipMemoryTypeHost with a device pointer) whose first and last bytes
// belong to the same allocation (the same range start; the runtime reports no range size above
// 2 GiB, so the last byte is asked instead) at consecutive device addresses.  nullptr otherwise
// (pageable memory, or a range past its allocation); len 0 asks nothing and gives nullptr.
uint8_t *mapped_host_range(const void *p, uint64_t len) {
    if (!p || !len) return nullptr;
    const void *last = static_cast<const uint8_t *>(p) + (len - 1);
    hipPointerAttribute_t a{}, b{};
    uint64_t start_a = 0, start_b = 0;
    const bool ok = hipPointerGetAttributes(&a, p) == hipSuccess && a.type == hipMemoryTypeHost && a.devicePointer &&
                    hipPointerGetAttributes(&b, last) == hipSuccess && b.type == hipMemoryTypeHost && b.devicePointer &&
                    hipPointerGetAttribute(&start_a, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR, (hipDeviceptr_t)p) ==
                        hipSuccess &&
                    hipPointerGetAttribute(&start_b, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR, (hipDeviceptr_t)last) ==
                        hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return nullptr;
    }
    uint8_t *dev = reinterpret_cast<uint8_t *>(a.devicePointer);
    if (start_a != start_b || reinterpret_cast<uint8_t *>(b.devicePointer) != dev + (len - 1)) return nullptr;
    return dev;
}

// Batches that move more host bytes than this (patterns, offsets and counts) are copied by the DMA
// engines even when they could be staged: at that size the copies' bandwidth wins, and staging
// kernels would take compute units from the counts in flight.
constexpr uint64_t STAGE_MAX_BYTES = 4ull << 20;

// The live free-memory reading is refreshed at most this often (a hipMemGetInfo call has been seen
// to block the loop for milliseconds).
constexpr double FREE_MEMORY_REFRESH_S = 5e-3;

struct Inflight {
    bool busy = false;
    uint64_t r0 = 0, r1 = 0, base = 0, nbytes = 0;
    uint32_t chunk = 0;
};

// Growth of the arena from the device's free memory: a new chunk holds max(need, budget) bytes,
// rounded up to 2 MiB, and is taken only while the free memory left after it stays at or above
// max(1 GiB, 1/64 of the device's memory).
constexpr uint64_t GROW_ROUND = 2ull << 20, GROW_MIN_HEADROOM = 1ull << 30;

}  // namespace

struct qr_server_s {
    int device;
    qr_quadfm fm;
    int slots;
    uint64_t budget, max_batch_patterns;
    uint32_t flags;
    int64_t last_staged = -1;  // batches of the last run staged by kernels (the rest were copied)
    std::vector<std::pair<uint8_t *, uint64_t>> chunks;  // the arena's device memory: the budget, then growth
    unsigned long long *heads;                            // one work-queue head per slot
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
};

namespace {

void release_server(qr_server_s *s) {
    if (!s) return;
    for (hipEvent_t e : s->events)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    for (const auto &c : s->chunks) (void)hipFree(c.first);
    if (s->heads) (void)hipFree(s->heads);
    delete s;
}

void drain(qr_server_s *s) {
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
}

// Adds a chunk of at least `need` bytes to the server and to the run's arena, if the device's free
// memory allows it (GROW_ROUND, GROW_MIN_HEADROOM); false leaves both unchanged.
bool grow_arena(qr_server_s *s, Arena &arena, uint64_t need) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uint64_t chunk = (std::max(need, s->budget) + GROW_ROUND - 1) / GROW_ROUND * GROW_ROUND;
    const uint64_t headroom = std::max<uint64_t>(GROW_MIN_HEADROOM, (uint64_t)tot / 64);
    if ((uint64_t)fr < chunk || (uint64_t)fr - chunk < headroom) return false;
    void *p = nullptr;
    if (hipMalloc(&p, chunk) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    s->chunks.push_back({reinterpret_cast<uint8_t *>(p), chunk});
    arena.add(chunk);
    return true;
}

}  // namespace

extern "C" {

int qr_server_create(qr_quadfm fm, int slots, uint64_t budget_bytes, uint64_t max_batch_patterns, uint32_t flags,
                     qr_server *out) {
    if (!out) return QR_EINVAL;
    *out = nullptr;
    if (!fm || slots < 1 || slots > 64 || budget_bytes < 4 * ALIGN || max_batch_patterns == 0 ||
        (flags & ~(QR_SERVE_CHECK_FREE_MEMORY | QR_SERVE_PACKED_PATTERNS | QR_SERVE_GROW_FROM_FREE_HBM |
                   QR_SERVE_COPY_ENGINE | QR_SERVE_BOTH_STRANDS))) {
        set_error("qr_server_create: need an index, 1..64 slots, a budget of at least 1 KiB and a batch cap");
        return QR_EINVAL;
    }
    qr_server_s *s = new (std::nothrow) qr_server_s{};
    if (!s) return QR_ENOMEM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return QR_EHIP;
    }
    s->fm = fm;
    s->slots = slots;
    s->budget = budget_bytes;
    s->max_batch_patterns = max_batch_patterns;
    s->flags = flags;
    s->streams.assign(slots, nullptr);
    s->events.assign(slots, nullptr);
    void *first = nullptr;
    const bool got = hipMalloc(&first, budget_bytes) == hipSuccess;
    if (got) s->chunks.push_back({reinterpret_cast<uint8_t *>(first), budget_bytes});
    if (!got || hipMalloc(&s->heads, 8 * (size_t)slots) != hipSuccess) {
        (void)hipGetLastError();
        release_server(s);
        set_error("qr_server_create: device allocation of %llu bytes failed", (unsigned long long)budget_bytes);
        return QR_ENOMEM;
    }
    for (int k = 0; k < slots; ++k) {
        if (hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->events[k], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            release_server(s);
            set_error("qr_server_create: stream or event creation failed");
            return QR_EHIP;
        }
    }
    *out = s;
    return QR_OK;
}

int64_t qr_server_last_run_staged(qr_server s) { return s ? s->last_staged : -1; }

uint64_t qr_server_arena_bytes(qr_server s) {
    uint64_t b = 0;
    if (s)
        for (const auto &c : s->chunks) b += c.second;
    return b;
}

int qr_server_free(qr_server s) {
    if (s) drain(s);
    release_server(s);
    return QR_OK;
}

int qr_server_run(qr_server s, const uint8_t *h_pat, const uint64_t *h_off, const uint64_t *h_req_off, uint64_t nreq,
                  const double *h_arrival_s, uint32_t *h_counts, double *h_finish_s, double deadline_s,
                  qr_serve_stats *stats) {
    if (!s || (nreq && (!h_off || !h_req_off || !h_arrival_s || !h_counts || !h_finish_s))) {
        set_error("qr_server_run: null server or array");
        return QR_EINVAL;
    }
    int rc = check_device(s->device);
    if (rc) return rc;
    for (uint64_t r = 0; r < nreq; ++r) {
        if (h_req_off[r + 1] < h_req_off[r] || (r && h_arrival_s[r] < h_arrival_s[r - 1])) {
            set_error("qr_server_run: request offsets and arrival times must be non-decreasing");
            return QR_EINVAL;
        }
    }
    if (nreq) {
        for (uint64_t p = h_req_off[0]; p < h_req_off[nreq]; ++p) {
            if (h_off[p + 1] < h_off[p]) {
                set_error("qr_server_run: pattern offsets must be non-decreasing (h_off[%llu] > h_off[%llu])",
                          (unsigned long long)p, (unsigned long long)(p + 1));
                return QR_EINVAL;
            }
        }
    }
    if (nreq && h_req_off[nreq] && !h_pat && h_off[h_req_off[nreq]] > h_off[h_req_off[0]]) {
        set_error("qr_server_run: h_pat is NULL");
        return QR_EINVAL;
    }
    const bool packed = s->flags & QR_SERVE_PACKED_PATTERNS;
    const uint32_t cflags = (s->flags & QR_SERVE_BOTH_STRANDS) ? QUADFM_BOTH_STRANDS : 0u;
    // a batch's pattern bytes at h_pat, from stream unit c0 (a byte, or a base of packed words) to c1:
    // bytes [c0 rounded down to 8, c1); packed, the whole words holding bases [c0, c1), from word c0 / 32
    auto pat_bytes = [&](uint64_t c0, uint64_t c1) -> uint64_t {
        if (!packed) return c1 > c0 ? c1 - c0 / 8 * 8 : 0;
        return c1 > c0 ? 8 * ((c1 + 31) / 32 - c0 / 32) : 0;
    };
    auto batch_bytes = [&](uint64_t r0, uint64_t r1) {
        const uint64_t p0 = h_req_off[r0], p1 = h_req_off[r1];
        return pad(pat_bytes(h_off[p0], h_off[p1])) + pad(8 * (p1 - p0 + 1)) + pad(4 * (p1 - p0)) + ALIGN;
    };
    const bool grow = s->flags & QR_SERVE_GROW_FROM_FREE_HBM;
    // Direct batches need every host range the run touches in pinned, device-mapped memory: h_pat
    // from byte 0 to the end of the last pattern (whole words when packed), the offsets and the counts.
    const uint8_t *dev_pat = nullptr, *dev_off = nullptr;
    uint8_t *dev_cnt = nullptr;
    uint64_t pat_end = 0;
    bool direct = false;
    if (nreq && !(s->flags & QR_SERVE_COPY_ENGINE)) {
        const uint64_t q0 = h_req_off[0], q1 = h_req_off[nreq], e = h_off[q1];
        pat_end = packed ? (e + 31) / 32 * 8 : e;
        dev_pat = mapped_host_range(h_pat, pat_end);
        dev_off = mapped_host_range(h_off + q0, 8 * (q1 - q0 + 1));
        dev_cnt = mapped_host_range(h_counts + q0, 4 * (q1 - q0));
        direct = (dev_pat || !pat_end) && dev_off && (dev_cnt || q1 == q0);
    }
    // Before the clock starts, on every slot's stream: a kernel, then a DMA read from each host array
    // the run may copy from, the pattern array's as large as a copied batch's.  The first copy that
    // follows kernels on a stream, reading a large host array, has been seen to hold the loop for
    // 5-9 ms; this pays that as setup instead of in the first copied batch.
    if (nreq) {
        const uint64_t q0 = h_req_off[0], q1 = h_req_off[nreq], e = h_off[q1];
        const uint64_t pat_all = packed ? (e + 31) / 32 * 8 : e;
        const uint64_t warm = std::min<uint64_t>({pat_all, STAGE_MAX_BYTES + (64u << 10), s->chunks[0].second});
        uint8_t *scratch = s->chunks[0].first;  // the arena is idle between runs
        hipError_t w = hipSuccess;
        for (int k = 0; k < s->slots && w == hipSuccess; ++k) {
            hipStream_t st = s->streams[k];
            hipLaunchKernelGGL(rebase_offsets, dim3(1), dim3(64), 0, st, reinterpret_cast<uint64_t *>(scratch), 0, 0);
            w = hipGetLastError();
            if (w == hipSuccess && h_pat && warm) w = hipMemcpyAsync(scratch, h_pat, warm, hipMemcpyHostToDevice, st);
            if (w == hipSuccess) w = hipMemcpyAsync(scratch, h_off + q0, 8, hipMemcpyHostToDevice, st);
            if (w == hipSuccess && q1 > q0) w = hipMemcpyAsync(scratch, h_counts + q0, 4, hipMemcpyHostToDevice, st);
        }
        for (int k = 0; k < s->slots && w == hipSuccess; ++k) w = hipStreamSynchronize(s->streams[k]);
        if (w != hipSuccess) {
            set_error("qr_server_run: %s", hipGetErrorString(w));
            return QR_EHIP;
        }
    }
    uint64_t staged = 0;
    double free_at = -1.0;  // time of the last free-memory reading
    size_t free_now = 0;
    Arena arena;
    for (const auto &c : s->chunks) arena.add(c.second);
    std::vector<Inflight> fl(s->slots);
    std::vector<int> free_slots;
    for (int k = s->slots - 1; k >= 0; --k) free_slots.push_back(k);
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    uint64_t nxt = 0, done = 0, batches = 0, reserved = 0, max_reserved = 0, inflight = 0, max_inflight = 0;
    int err = QR_OK;
    while (done < nreq) {
        const double now = elapsed();
        if (now > deadline_s) {
            set_error("qr_server_run: deadline of %.1f s passed with %llu of %llu requests done", deadline_s,
                      (unsigned long long)done, (unsigned long long)nreq);
            err = QR_ERANGE;
            break;
        }
        bool progressed = false;
        // completions, in any order
        for (int k = 0; k < s->slots; ++k) {
            if (!fl[k].busy) continue;
            const hipError_t q = hipEventQuery(s->events[k]);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                set_error("qr_server_run: %s", hipGetErrorString(q));
                err = QR_EHIP;
                break;
            }
            const double t = elapsed();
            for (uint64_t r = fl[k].r0; r < fl[k].r1; ++r) h_finish_s[r] = t;
            done += fl[k].r1 - fl[k].r0;
            arena.release(fl[k].chunk, fl[k].base, fl[k].nbytes);
            reserved -= fl[k].nbytes;
            fl[k].busy = false;
            --inflight;
            free_slots.push_back(k);
            progressed = true;
        }
        if (err) break;
        // admissions: every arrived request, FIFO, in one batch per free slot
        while (!free_slots.empty() && nxt < nreq && h_arrival_s[nxt] <= now) {
            const uint64_t arrived =
                (uint64_t)(std::upper_bound(h_arrival_s + nxt, h_arrival_s + nreq, now) - h_arrival_s);
            uint64_t r1 = nxt + 1;
            while (r1 < arrived && h_req_off[r1 + 1] - h_req_off[nxt] <= s->max_batch_patterns) ++r1;
            uint64_t nb = batch_bytes(nxt, r1);
            while (r1 > nxt + 1 && nb > s->budget) nb = batch_bytes(nxt, --r1);
            if (nb > arena.largest() && !(grow && grow_arena(s, arena, nb))) {
                if (grow)
                    set_error("qr_server_run: request %llu needs %llu bytes, more than the arena's largest chunk %llu, "
                              "and the device's free memory leaves no room for a chunk that large",
                              (unsigned long long)nxt, (unsigned long long)nb, (unsigned long long)arena.largest());
                else
                    set_error("qr_server_run: request %llu needs %llu bytes, more than the budget %llu",
                              (unsigned long long)nxt, (unsigned long long)nb, (unsigned long long)s->budget);
                err = QR_ERANGE;
                break;
            }
            if (s->flags & QR_SERVE_CHECK_FREE_MEMORY) {
                if (free_at < 0 || now - free_at > FREE_MEMORY_REFRESH_S) {
                    size_t tot = 0;
                    if (hipMemGetInfo(&free_now, &tot) != hipSuccess) {
                        (void)hipGetLastError();
                        free_now = 0;
                    }
                    free_at = now;
                }
                if (nb > free_now) break;
            }
            uint32_t ck = 0;
            uint64_t base = 0;
            // no room: grow the arena if allowed, else wait for a batch to finish
            if (!arena.alloc(nb, ck, base) && !(grow && grow_arena(s, arena, nb) && arena.alloc(nb, ck, base))) break;
            const int k = free_slots.back();
            free_slots.pop_back();
            const uint64_t p0 = h_req_off[nxt], p1 = h_req_off[r1], npat = p1 - p0;
            const uint64_t c0 = h_off[p0], chars = pat_bytes(c0, h_off[p1]);
            const uint64_t first = packed ? c0 / 32 * 8 : c0 / 8 * 8;     // first byte of h_pat the batch copies
            const uint64_t rebase = packed ? c0 / 32 * 32 : c0 / 8 * 8;  // stream unit of that byte
            uint8_t *d_pat = s->chunks[ck].first + base;
            uint64_t *d_off = reinterpret_cast<uint64_t *>(d_pat + pad(chars));
            uint32_t *d_cnt = reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(d_off) + pad(8 * (npat + 1)));
            hipStream_t st = s->streams[k];
            hipError_t e = hipSuccess;
            const bool stage = direct && chars + 12 * npat + 8 <= STAGE_MAX_BYTES;
            staged += stage;
            if (stage) {
                if (chars && first + chars > pat_end) {  // cannot happen: offsets are non-decreasing
                    set_error("qr_server_run: batch pattern bytes beyond the checked host range");
                    err = QR_EINVAL;
                    break;
                }
                const uint64_t *so = reinterpret_cast<const uint64_t *>(dev_off) + (p0 - h_req_off[0]);
                hipLaunchKernelGGL(stage_in, dim3(stage_blocks(std::max(chars / 8, npat + 1))), dim3(256), 0, st, d_pat,
                                   chars ? dev_pat + first : nullptr, chars, d_off, so, npat + 1, rebase);
                e = hipGetLastError();
            } else {
                if (chars) e = hipMemcpyAsync(d_pat, h_pat + first, chars, hipMemcpyHostToDevice, st);
                if (e == hipSuccess) e = hipMemcpyAsync(d_off, h_off + p0, 8 * (npat + 1), hipMemcpyHostToDevice, st);
                if (e == hipSuccess) {
                    hipLaunchKernelGGL(rebase_offsets, dim3((uint32_t)((npat + 1 + 255) / 256)), dim3(256), 0, st,
                                       d_off, npat + 1, rebase);
                    e = hipGetLastError();
                }
            }
            if (e != hipSuccess) {
                set_error("qr_server_run: %s", hipGetErrorString(e));
                err = QR_EHIP;
                break;
            }
            rc = packed ? quadfm_count_packed(s->fm, reinterpret_cast<const uint64_t *>(d_pat), chars / 8 * 32, d_off,
                                              npat, cflags, d_cnt, s->heads + k, st)
                        : quadfm_count_ex(s->fm, d_pat, chars, d_off, npat, cflags, d_cnt, s->heads + k, st);
            if (rc) {
                err = rc;
                break;
            }
            if (stage) {
                if (npat) {
                    uint32_t *dc = reinterpret_cast<uint32_t *>(dev_cnt) + (p0 - h_req_off[0]);
                    hipLaunchKernelGGL(stage_out, dim3(stage_blocks(npat)), dim3(256), 0, st, dc, d_cnt, npat);
                }
                e = hipGetLastError();
            } else {
                e = hipMemcpyAsync(h_counts + p0, d_cnt, 4 * npat, hipMemcpyDeviceToHost, st);
            }
            if (e == hipSuccess) e = hipEventRecord(s->events[k], st);
            if (e != hipSuccess) {
                set_error("qr_server_run: %s", hipGetErrorString(e));
                err = QR_EHIP;
                break;
            }
            fl[k] = Inflight{true, nxt, r1, base, nb, ck};
            reserved += nb;
            max_reserved = std::max(max_reserved, reserved);
            ++inflight;
            max_inflight = std::max(max_inflight, inflight);
            ++batches;
            nxt = r1;
            progressed = true;
        }
        if (err) break;
        if (!progressed) {
            // nothing to do until an arrival or a completion: poll again shortly
            const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(2);
            while (std::chrono::steady_clock::now() < until) {
            }
        }
    }
    s->last_staged = (int64_t)staged;
    drain(s);  // no copy may still target the caller's buffers on return
    if (stats) {
        stats->batches = batches;
        stats->max_inflight = max_inflight;
        stats->max_reserved_bytes = max_reserved;
        stats->wall_s = elapsed();
    }
    return err;
}

}  // extern "C"
