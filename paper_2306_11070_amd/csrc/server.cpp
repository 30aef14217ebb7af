// Request server: admission against a device-memory budget, resident
// compressed streams, and continuous batching of waiting requests into
// batch plans that run concurrently on a few streams.
//
// One scheduler thread does all device work.  Each turn it
//   1. retires the batches whose completion event has fired (statuses and
//      stream lengths come back in one pinned copy per batch), and
//   2. while a launch slot (stream) is free and requests wait, takes waiting
//      requests in arrival order for as long as their memory fits the
//      budget, builds one batch from them (a compress plan and a decode
//      plan, tables in the arena, uploaded from pinned staging), and queues
//      it on the slot's stream.
// Requests submitted while batches run therefore join the next batch as soon
// as a slot frees up; batches on different slots overlap on the device.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace huff;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr uint64_t kAlign = 256;
inline uint64_t up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over one device allocation; offsets are kAlign-aligned
// and free ranges are kept coalesced.
class Arena {
public:
    bool init(uint64_t bytes) {
        size_ = up(bytes, kAlign);
        if (hipMalloc(&base_, size_) != hipSuccess) return false;
        free_[0] = size_;
        return true;
    }
    void destroy() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    bool alloc(uint64_t bytes, uint64_t& off) {
        bytes = up(std::max<uint64_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = up(std::max<uint64_t>(bytes, 1), kAlign);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint8_t* at(uint64_t off) const { return base_ + off; }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

private:
    uint8_t* base_ = nullptr;
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

// A compressed stream or a decode output held in the arena.
struct Resident {
    uint64_t off = 0, bytes = 0;  // arena block
    uint64_t n = 0, total_bits = 0;
    bool is_output = false;       // decode output (bytes at `out`) rather than a compressed stream
    huff_dcb* cb = nullptr;
    uint32_t* words = nullptr;
    uint64_t nwords = 0;
    uint64_t* chunk_off = nullptr;
    uint32_t* sub_lo = nullptr;
    uint8_t* out = nullptr;
    uint32_t readers = 0;         // queued or running decodes of this stream
    bool released = false;        // free once readers drop to 0
};

struct Req {
    uint64_t ticket = 0;
    huff_request r{};
    huff_result res{};
    bool done = false;
    uint64_t block_off = 0, block_bytes = 0;  // its arena block (stream or output)
    uint64_t handle = 0;                      // resident made for it
    uint64_t src = 0;                         // decode: stream read
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* staging = nullptr;   // pinned: tables going up
    uint64_t staging_bytes = 0;
    void* readback = nullptr;  // pinned: statuses and lengths coming back
    uint64_t readback_bytes = 0;
    bool busy = false;
    std::vector<Req*> reqs;
    uint64_t tables_off = 0, tables_bytes = 0;
    uint32_t ncomp = 0;
};

bool grow_pinned(void*& p, uint64_t& have, uint64_t need) {
    if (have >= need) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    have = 0;
    const uint64_t sz = up(std::max<uint64_t>(need, 1 << 16), 1 << 16);
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return false;
    have = sz;
    return true;
}

}  // namespace

struct huff_server {
    huff_ctx* ctx = nullptr;
    huff_server_cfg cfg{};
    Arena arena;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> waiting;
    std::unordered_map<uint64_t, Req*> reqs;          // by ticket
    std::unordered_map<uint64_t, Resident> residents;  // by handle
    uint64_t next_ticket = 1, next_handle = 1;
    uint64_t batches = 0, completed = 0;
    bool stop = false;
    std::thread worker;

    uint64_t stream_bytes(uint64_t n) const {
        const uint64_t nch = (n + cfg.chunk_size - 1) / cfg.chunk_size;
        const uint64_t nsub = cfg.sub_size ? (n + cfg.sub_size - 1) / cfg.sub_size : 0;
        // Huffman codes average fewer than H + 1 <= 9 bits per byte (and 1 bit
        // with a single symbol): 9 bits per byte always holds the stream.
        const uint64_t words = (9 * n + 31) / 32 + 4;
        return up(sizeof(huff_dcb), kAlign) + up(words * 4, kAlign) + up((nch + 1) * 8, kAlign) +
               up((cfg.sub_size ? nsub + 1 : 1) * 4, kAlign);
    }
    uint64_t tables_bytes(uint32_t nreq, uint64_t ntiles) const {
        return 2 * up(std::max<uint32_t>(nreq, 1) * sizeof(FileDesc), kAlign) + up(nreq * 4 + 8, kAlign) +
               up(nreq * 8 + 8, kAlign) + up(nreq * 8 + 8, kAlign) + up(std::max<uint64_t>(ntiles, 1) * 4, kAlign) +
               up(std::max<uint32_t>(nreq, 1) * sizeof(CmpJob), kAlign) +
               up(batch_workspace_bytes(ntiles) + 4 * kAlign, kAlign) + up(std::max<uint32_t>(nreq, 1) * 2048, kAlign);
    }

    void run();
    bool launch(Slot& sl);
    void retire(Slot& sl);
    void free_resident(uint64_t h) {
        auto it = residents.find(h);
        if (it == residents.end()) return;
        arena.release(it->second.off, it->second.bytes);
        residents.erase(it);
    }
};

// Builds one batch from waiting requests and queues it on the slot's stream.
// Called with the lock held.  Returns false if nothing could be launched.
bool huff_server::launch(Slot& sl) {
    std::vector<Req*> take;
    uint64_t ntiles = 0;
    // admission in arrival order while memory lasts (the batch tables are
    // sized for what is taken and allocated last)
    while (!waiting.empty() && take.size() < cfg.max_batch) {
        Req* q = waiting.front();
        uint64_t need;
        if (q->r.op == HUFF_OP_COMPRESS) need = stream_bytes(q->r.n);
        else need = up(std::max<uint64_t>(residents[q->src].n, 1), kAlign);
        uint64_t off;
        if (!arena.alloc(need, off)) break;
        q->block_off = off;
        q->block_bytes = need;
        take.push_back(q);
        waiting.pop_front();
        if (q->r.op == HUFF_OP_COMPRESS) ntiles += (q->r.n + kEncTile - 1) / kEncTile;
    }
    if (take.empty()) return false;
    uint64_t toff;
    const uint64_t tbytes = tables_bytes((uint32_t)take.size(), ntiles);
    while (!arena.alloc(tbytes, toff)) {
        // give the last request back and retry with fewer (the first one
        // always fits: submit checked it against the whole budget)
        Req* q = take.back();
        take.pop_back();
        arena.release(q->block_off, q->block_bytes);
        waiting.push_front(q);
        if (take.empty()) return false;
        ntiles = 0;
        for (Req* t : take)
            if (t->r.op == HUFF_OP_COMPRESS) ntiles += (t->r.n + kEncTile - 1) / kEncTile;
    }
    const double t0 = now_s();
    // file lists of the two plans; statuses and lengths in the tables block
    std::vector<huff_file> cf, df;
    std::vector<Req*> creq, dreq;
    const uint32_t nreq = (uint32_t)take.size();
    uint8_t* tb = arena.at(toff);
    uint64_t cur = 0;
    auto carve = [&](uint64_t bytes) {
        uint8_t* p = tb + cur;
        cur += up(bytes, kAlign);
        return p;
    };
    FileDesc* d_enc = (FileDesc*)carve(std::max<uint32_t>(nreq, 1) * sizeof(FileDesc));
    FileDesc* d_dec = (FileDesc*)carve(std::max<uint32_t>(nreq, 1) * sizeof(FileDesc));
    int32_t* d_status = (int32_t*)carve(nreq * 4 + 8);
    const uint64_t** d_lenptr = (const uint64_t**)carve(nreq * 8 + 8);
    uint64_t* d_len = (uint64_t*)carve(nreq * 8 + 8);
    uint32_t* d_tile_file = (uint32_t*)carve(std::max<uint64_t>(ntiles, 1) * 4);
    CmpJob* d_jobs = (CmpJob*)carve(std::max<uint32_t>(nreq, 1) * sizeof(CmpJob));
    uint8_t* ws = carve(batch_workspace_bytes(ntiles) + 4 * kAlign);
    unsigned long long* d_file_hist = (unsigned long long*)carve(std::max<uint32_t>(nreq, 1) * 2048);
    for (uint32_t i = 0; i < nreq; ++i) {
        Req* q = take[i];
        q->res.t_start = t0;
        huff_file f;
        memset(&f, 0, sizeof(f));
        f.status = d_status + i;
        if (q->r.op == HUFF_OP_COMPRESS) {
            Resident rs;
            rs.off = q->block_off;
            rs.bytes = q->block_bytes;
            rs.n = q->r.n;
            uint8_t* p = arena.at(q->block_off);
            const uint64_t n = q->r.n;
            const uint64_t nch = (n + cfg.chunk_size - 1) / cfg.chunk_size;
            const uint64_t nsub = cfg.sub_size ? (n + cfg.sub_size - 1) / cfg.sub_size : 0;
            rs.cb = (huff_dcb*)p;
            p += up(sizeof(huff_dcb), kAlign);
            rs.words = (uint32_t*)p;
            rs.nwords = (9 * n + 31) / 32 + 4;
            p += up(rs.nwords * 4, kAlign);
            rs.chunk_off = (uint64_t*)p;
            p += up((nch + 1) * 8, kAlign);
            rs.sub_lo = cfg.sub_size ? (uint32_t*)p : nullptr;
            (void)nsub;
            f.in = q->r.d_in;
            f.n = n;
            f.cb = rs.cb;
            f.words = rs.words;
            f.cap_words = rs.nwords;
            f.chunk_off = rs.chunk_off;
            f.sub_lo = rs.sub_lo;
            q->handle = next_handle++;
            residents[q->handle] = rs;
            cf.push_back(f);
            creq.push_back(q);
        } else {
            Resident& src = residents[q->src];
            Resident out;
            out.off = q->block_off;
            out.bytes = q->block_bytes;
            out.n = src.n;
            out.is_output = true;
            out.out = arena.at(q->block_off);
            f.n = src.n;
            f.cb = src.cb;
            f.words = src.words;
            f.cap_words = src.nwords;
            f.chunk_off = src.chunk_off;
            f.sub_lo = src.sub_lo;
            f.out = out.out;
            q->handle = next_handle++;
            residents[q->handle] = out;
            df.push_back(f);
            dreq.push_back(q);
        }
    }
    // order the requests as the readback is laid out: compress first
    sl.reqs.clear();
    sl.reqs.insert(sl.reqs.end(), creq.begin(), creq.end());
    sl.reqs.insert(sl.reqs.end(), dreq.begin(), dreq.end());
    for (uint32_t i = 0; i < nreq; ++i) {
        if (i < cf.size()) cf[i].status = d_status + i;
        else df[i - cf.size()].status = d_status + i;
    }
    sl.ncomp = (uint32_t)cf.size();
    sl.tables_off = toff;
    sl.tables_bytes = tbytes;

    BatchTables ct, dt;
    huff_status st = batch_tables(cf.data(), (uint32_t)cf.size(), cfg.chunk_size, cfg.sub_size, ct);
    if (st == HUFF_OK) st = batch_tables(df.data(), (uint32_t)df.size(), cfg.chunk_size, cfg.sub_size, dt, true);
    // result checks of the requests that carry an expected result
    std::vector<CmpJob> jobs;
    uint32_t cmp_blocks = 0;
    for (uint32_t i = 0; i < nreq; ++i) {
        const Req* q = sl.reqs[i];
        if (!q->r.d_expect) continue;
        CmpJob j;
        memset(&j, 0, sizeof(j));
        j.want = (const uint8_t*)q->r.d_expect;
        j.status = d_status + i;
        const Resident& rs = residents[q->handle];
        if (q->r.op == HUFF_OP_COMPRESS) {
            const uint64_t nch = (rs.n + cfg.chunk_size - 1) / cfg.chunk_size;
            j.got = (const uint8_t*)rs.words;
            j.bytes = (q->r.expect_bits + 31) / 32 * 4;
            if (j.bytes > rs.nwords * 4) j.bytes = rs.nwords * 4;  // a longer expectation fails on the length
            j.got_bits = rs.chunk_off + nch;
            j.want_bits = q->r.expect_bits;
        } else {
            j.got = rs.out;
            j.bytes = rs.n;
        }
        j.first_block = cmp_blocks;
        j.nblocks = compare_blocks(j.bytes);
        cmp_blocks += j.nblocks;
        jobs.push_back(j);
    }
    // staging: [enc | dec | status zeros | length pointers | tile_file | checks]
    const uint64_t sz_enc = cf.size() * sizeof(FileDesc), sz_dec = df.size() * sizeof(FileDesc);
    const uint64_t o_stat = sz_enc + sz_dec, o_lp = o_stat + up(nreq * 4, 8), o_tf = o_lp + cf.size() * 8;
    const uint64_t o_jobs = up(o_tf + ct.ntiles * 4, 8);
    const uint64_t need = o_jobs + jobs.size() * sizeof(CmpJob);
    if (st == HUFF_OK && !grow_pinned(sl.staging, sl.staging_bytes, need)) st = HUFF_E_NOMEM;
    if (st == HUFF_OK && !grow_pinned(sl.readback, sl.readback_bytes, nreq * 4 + cf.size() * 8 + 16)) st = HUFF_E_NOMEM;
    if (st == HUFF_OK) {
        uint8_t* h = (uint8_t*)sl.staging;
        memcpy(h, ct.enc.data(), sz_enc);
        memcpy(h + sz_enc, dt.dec.data(), sz_dec);
        memset(h + o_stat, 0, nreq * 4);
        const uint64_t** lp = (const uint64_t**)(h + o_lp);
        for (size_t i = 0; i < cf.size(); ++i) {
            const uint64_t nch = (cf[i].n + cfg.chunk_size - 1) / cfg.chunk_size;
            lp[i] = cf[i].chunk_off + nch;
        }
        memcpy(h + o_tf, ct.tile_file.data(), ct.ntiles * 4);
        if (!jobs.empty()) memcpy(h + o_jobs, jobs.data(), jobs.size() * sizeof(CmpJob));
        hipStream_t s = sl.stream;
        bool ok = true;
        if (sz_enc) ok = ok && hipMemcpyAsync(d_enc, h, sz_enc, hipMemcpyHostToDevice, s) == hipSuccess;
        if (sz_dec) ok = ok && hipMemcpyAsync(d_dec, h + sz_enc, sz_dec, hipMemcpyHostToDevice, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(d_status, h + o_stat, nreq * 4, hipMemcpyHostToDevice, s) == hipSuccess;
        if (cf.size())
            ok = ok && hipMemcpyAsync(d_lenptr, lp, cf.size() * 8, hipMemcpyHostToDevice, s) == hipSuccess;
        if (ct.ntiles)
            ok = ok && hipMemcpyAsync(d_tile_file, h + o_tf, ct.ntiles * 4, hipMemcpyHostToDevice, s) == hipSuccess;
        if (!jobs.empty())
            ok = ok && hipMemcpyAsync(d_jobs, h + o_jobs, jobs.size() * sizeof(CmpJob), hipMemcpyHostToDevice, s) ==
                           hipSuccess;
        if (!ok) st = HUFF_E_HIP;
        // the two plans over the tables block
        huff_batch pc, pd;
        pc.ctx = pd.ctx = ctx;
        pc.device = pd.device = ctx->device;
        pc.owns = pd.owns = false;
        pc.chunk_size = pd.chunk_size = cfg.chunk_size;
        pc.sub_size = pd.sub_size = cfg.sub_size;
        pc.nfiles = (uint32_t)cf.size();
        pc.ntiles = ct.ntiles;
        pc.d_enc = d_enc;
        pc.d_tile_file = d_tile_file;
        const uint64_t nblk = ct.ntiles / kScanTilesPerBlock + 1;
        uint8_t* w = ws;
        pc.d_tile_hist = (uint16_t*)w;
        w += up(std::max<uint64_t>(ct.ntiles, 1) * 512, kAlign);
        pc.d_tile_local = (uint32_t*)w;
        w += up(std::max<uint64_t>(ct.ntiles, 1) * 4, kAlign);
        pc.d_blk_tail = (unsigned long long*)w;
        w += up(nblk * 8, kAlign);
        pc.d_blk_carry = (unsigned long long*)w;
        pc.d_file_hist = d_file_hist;  // [nfiles][256] totals
        pd.nfiles = (uint32_t)df.size();
        pd.nitems = dt.nitems;
        pd.can_decode = dt.can_decode;
        pc.aligned = ct.aligned;
        pd.d_dec = d_dec;
        if (st == HUFF_OK && pc.nfiles) st = batch_launch(&pc, HUFF_OP_COMPRESS, s);
        if (st == HUFF_OK && pc.nfiles) st = hip_status(launch_gather_u64(d_lenptr, d_len, pc.nfiles, s));
        if (st == HUFF_OK && pd.nfiles) st = batch_launch(&pd, HUFF_OP_DECODE, s);
        if (st == HUFF_OK && !jobs.empty())
            st = hip_status(launch_compare(d_jobs, (uint32_t)jobs.size(), cmp_blocks, s));
        uint8_t* rb = (uint8_t*)sl.readback;
        if (st == HUFF_OK && hipMemcpyAsync(rb, d_status, nreq * 4, hipMemcpyDeviceToHost, s) != hipSuccess) st = HUFF_E_HIP;
        if (st == HUFF_OK && cf.size() &&
            hipMemcpyAsync(rb + up(nreq * 4, 8), d_len, cf.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = HUFF_E_HIP;
        if (st == HUFF_OK && hipEventRecord(sl.done, s) != hipSuccess) st = HUFF_E_HIP;
    }
    if (st != HUFF_OK) {
        // nothing usable was queued: fail these requests now
        (void)hipStreamSynchronize(sl.stream);
        const double t = now_s();
        for (Req* q : sl.reqs) {
            q->res.status = st;
            q->res.t_done = t;
            q->done = true;
            free_resident(q->handle);
            q->handle = 0;
            if (q->r.op == HUFF_OP_DECODE) {
                Resident& src = residents[q->src];
                if (--src.readers == 0 && src.released) free_resident(q->src);
            }
            ++completed;
        }
        arena.release(sl.tables_off, sl.tables_bytes);
        sl.reqs.clear();
        cv_done.notify_all();
        return true;
    }
    sl.busy = true;
    ++batches;
    return true;
}

// Completes the slot's batch (its event has fired).  Lock held.
void huff_server::retire(Slot& sl) {
    const double t = now_s();
    const uint8_t* rb = (const uint8_t*)sl.readback;
    const uint32_t nreq = (uint32_t)sl.reqs.size();
    const int32_t* stat = (const int32_t*)rb;
    const uint64_t* len = (const uint64_t*)(rb + up(nreq * 4, 8));
    for (uint32_t i = 0; i < nreq; ++i) {
        Req* q = sl.reqs[i];
        q->res.status = stat[i];
        q->res.t_done = t;
        q->res.handle = q->handle;
        if (q->r.op == HUFF_OP_COMPRESS) {
            Resident& rs = residents[q->handle];
            rs.total_bits = len[i];
            q->res.in_bytes = q->r.n;
            q->res.out_bytes = (len[i] + 7) / 8;
        } else {
            Resident& src = residents[q->src];
            q->res.in_bytes = (src.total_bits + 7) / 8;
            q->res.out_bytes = src.n;
            if (--src.readers == 0 && src.released) free_resident(q->src);
        }
        if (stat[i] != HUFF_OK || (q->r.flags & HUFF_REQ_DISCARD)) {  // keeps nothing
            free_resident(q->handle);
            q->res.handle = 0;
        }
        q->done = true;
        ++completed;
    }
    arena.release(sl.tables_off, sl.tables_bytes);
    sl.reqs.clear();
    sl.busy = false;
    cv_done.notify_all();
}

void huff_server::run() {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = false;
        for (Slot& sl : slots)
            if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
                retire(sl);
                progress = true;
            }
        for (Slot& sl : slots)
            if (!sl.busy && !waiting.empty() && launch(sl)) progress = true;
        bool busy = false;
        for (Slot& sl : slots) busy = busy || sl.busy;
        if (stop && !busy && !progress && !waiting.empty()) {
            // shutting down with requests that cannot be admitted: fail them
            const double t = now_s();
            for (Req* q : waiting) {
                q->res.status = HUFF_E_NOMEM;
                q->res.t_done = t;
                q->done = true;
                if (q->r.op == HUFF_OP_DECODE) {
                    Resident& src = residents[q->src];
                    if (--src.readers == 0 && src.released) free_resident(q->src);
                }
            }
            waiting.clear();
            cv_done.notify_all();
        }
        if (stop && !busy && waiting.empty()) break;
        if (!progress) {
            if (busy) {
                // a batch is on the device: poll its event often
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }
}

extern "C" {

huff_status huff_server_create(huff_ctx* ctx, const huff_server_cfg* cfg, huff_server** out) {
    if (!out) return HUFF_E_INVAL;
    *out = nullptr;
    if (!ctx) return HUFF_E_INVAL;
    huff_server_cfg c = cfg ? *cfg : huff_server_cfg{};
    if (!c.mem_budget_bytes) c.mem_budget_bytes = 1ull << 30;
    if (!c.nslots) c.nslots = 2;
    if (!c.max_batch) c.max_batch = 512;
    if (!c.chunk_size) c.chunk_size = 256u << 10;
    if (c.nslots > 16 || !is_pow2(c.chunk_size) || c.chunk_size < 1024 || c.chunk_size > (64u << 20)) return HUFF_E_INVAL;
    if (c.sub_size && (!is_pow2(c.sub_size) || c.sub_size < 16 || c.sub_size > c.chunk_size)) return HUFF_E_INVAL;
    DeviceGuard g(ctx->device);
    huff_server* s = new (std::nothrow) huff_server();
    if (!s) return HUFF_E_NOMEM;
    s->ctx = ctx;
    s->cfg = c;
    if (!s->arena.init(c.mem_budget_bytes)) {
        delete s;
        return HUFF_E_NOMEM;
    }
    s->slots.resize(c.nslots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            huff_server_destroy(s);
            return HUFF_E_HIP;
        }
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return HUFF_OK;
}

huff_status huff_server_submit(huff_server* s, const huff_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return HUFF_E_INVAL;
    Req* q = new (std::nothrow) Req();
    if (!q) return HUFF_E_NOMEM;
    q->r = *req;
    q->res.t_submit = now_s();
    q->res.status = HUFF_E_AGAIN;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) { delete q; return HUFF_E_INVAL; }
    uint64_t need;
    if (req->op == HUFF_OP_COMPRESS) {
        if (req->n >= kMaxN || (req->n && !req->d_in)) { delete q; return HUFF_E_INVAL; }
        need = s->stream_bytes(req->n);
        const uint64_t nt = (req->n + kEncTile - 1) / kEncTile;
        need += s->tables_bytes(1, nt);
    } else if (req->op == HUFF_OP_DECODE) {
        auto it = s->residents.find(req->stream_handle);
        if (it == s->residents.end() || it->second.is_output || it->second.released) { delete q; return HUFF_E_NOTFOUND; }
        need = up(std::max<uint64_t>(it->second.n, 1), kAlign) + s->tables_bytes(1, 0);
        it->second.readers++;
        q->src = req->stream_handle;
    } else {
        delete q;
        return HUFF_E_INVAL;
    }
    if (need > s->arena.size()) {
        if (req->op == HUFF_OP_DECODE) s->residents[q->src].readers--;
        delete q;
        return HUFF_E_NOMEM;
    }
    q->ticket = s->next_ticket++;
    s->reqs[q->ticket] = q;
    s->waiting.push_back(q);
    *ticket = q->ticket;
    s->cv_work.notify_one();
    return HUFF_OK;
}

huff_status huff_server_poll(huff_server* s, uint64_t ticket, huff_result* out) {
    if (!s || !out) return HUFF_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return HUFF_E_NOTFOUND;
    if (!it->second->done) return HUFF_E_AGAIN;
    *out = it->second->res;
    delete it->second;
    s->reqs.erase(it);
    return HUFF_OK;
}

huff_status huff_server_wait(huff_server* s, uint64_t ticket, huff_result* out) {
    if (!s || !out) return HUFF_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return HUFF_E_NOTFOUND;
    Req* q = it->second;
    s->cv_done.wait(lk, [q] { return q->done; });
    *out = q->res;
    s->reqs.erase(ticket);
    delete q;
    return HUFF_OK;
}

huff_status huff_server_stream(huff_server* s, uint64_t handle, huff_stream_info* out) {
    if (!s || !out) return HUFF_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->residents.find(handle);
    if (it == s->residents.end() || it->second.released) return HUFF_E_NOTFOUND;
    const Resident& r = it->second;
    out->n = r.n;
    out->total_bits = r.total_bits;
    out->cb = r.cb;
    out->words = r.words;
    out->chunk_off = r.chunk_off;
    out->sub_lo = r.sub_lo;
    out->out = r.out;
    return HUFF_OK;
}

huff_status huff_server_release(huff_server* s, uint64_t handle) {
    if (!s) return HUFF_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->residents.find(handle);
    if (it == s->residents.end() || it->second.released) return HUFF_E_NOTFOUND;
    if (it->second.readers) {
        it->second.released = true;  // freed by the last decode that reads it
        return HUFF_OK;
    }
    s->free_resident(handle);
    return HUFF_OK;
}

huff_status huff_server_replay(huff_server* s, const huff_request* reqs, const double* arrival_s, uint32_t count,
                               huff_result* results) {
    if (!s || (count && (!reqs || !arrival_s || !results))) return HUFF_E_INVAL;
    std::vector<uint64_t> tickets(count, 0);
    std::vector<huff_status> sub(count, HUFF_OK);
    const double t0 = now_s();
    for (uint32_t i = 0; i < count; ++i) {
        while (now_s() - t0 < arrival_s[i]) {
        }
        sub[i] = huff_server_submit(s, &reqs[i], &tickets[i]);
    }
    for (uint32_t i = 0; i < count; ++i) {
        if (sub[i] != HUFF_OK) {
            memset(&results[i], 0, sizeof(results[i]));
            results[i].status = sub[i];
        } else {
            const huff_status st = huff_server_wait(s, tickets[i], &results[i]);
            if (st != HUFF_OK) results[i].status = st;
        }
        results[i].t_submit = t0 + arrival_s[i];  // open loop: latency from the scheduled arrival
    }
    return HUFF_OK;
}

huff_status huff_server_stats(huff_server* s, uint64_t out[6]) {
    if (!s || !out) return HUFF_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->batches;
    out[1] = s->completed;
    out[2] = s->arena.used();
    out[3] = s->arena.peak();
    out[4] = s->waiting.size();
    uint64_t busy = 0;
    for (const Slot& sl : s->slots) busy += sl.busy ? 1 : 0;
    out[5] = busy;
    return HUFF_OK;
}

void huff_server_destroy(huff_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    DeviceGuard g(s->ctx->device);
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.readback) (void)hipHostFree(sl.readback);
    }
    for (auto& kv : s->reqs) delete kv.second;
    s->arena.destroy();
    delete s;
}

}  // extern "C"
