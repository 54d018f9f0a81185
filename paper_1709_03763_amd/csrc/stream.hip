// Memory-capped streaming of voxel blocks between the GPU and the host
// (Sec. 3, "SDF volume": only the blocks near the camera are kept in GPU
// memory, the others are streamed to the host; Sec. 4.3: before a
// re-integration the blocks around the poses it works at are streamed in).
//
// The device pool holds at most max_blocks blocks.  sc_stream_out moves
// every block whose centre lies outside a sphere to a host store and
// compacts the pool; in streaming mode every operation (plain or batched)
// first streams in, from the host store, exactly those of its candidate
// blocks that the store holds, so each operation sees every block it can
// touch and the field equals the one a fully resident volume would hold,
// bit for bit, whatever sphere the caller streams to.  The sphere decides
// only how much stays on the device between calls.
#include <string.h>

#include <algorithm>
#include <new>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "kernels.hpp"

// Host side of the streaming mode: where each host-held block lives, the
// host copies, and pinned / device staging for the transfers.
struct StreamStore {
    bool enabled = false;
    size_t block_bytes = 0;                      // one block's record in the pool
    std::unordered_map<uint64_t, size_t> where;  // block key -> host slot
    std::vector<unsigned char> arena;            // host slots x block_bytes
    std::vector<size_t> free_slots;
    size_t n_slots = 0;
    unsigned char* h_stage = nullptr;  // pinned, blocks
    unsigned char* d_stage = nullptr;  // device, blocks
    size_t stage_cap = 0;              // blocks
    uint64_t* h_keys = nullptr;        // pinned
    uint64_t* d_keys = nullptr;        // device: requested keys
    uint64_t* d_all = nullptr;         // device: every candidate key of the operation or chunk
    int32_t* d_slots = nullptr;        // device
    int32_t* h_slots = nullptr;        // pinned
    size_t keys_cap = 0;
    uint32_t* d_req = nullptr;         // device counter
    int64_t blocks_out = 0, blocks_in = 0;
};

namespace sc {

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------

// Inserts (key, slot) into the block hash (the key is absent).
__device__ inline void hash_put(const VolDev& v, uint64_t key, int slot)
{
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    uint32_t h = hash_block(bx, by, bz) & v.bucket_mask;
    for (uint32_t probe = 0; probe <= v.bucket_mask; ++probe) {
        const uint64_t old =
            atomicCAS((unsigned long long*)(v.keys + h), (unsigned long long)kKeyEmpty, (unsigned long long)key);
        if (old == kKeyEmpty) {
            v.vals[h] = slot;
            return;
        }
        h = (h + 1) & v.bucket_mask;
    }
    set_error(v.err, SC_EHASHFULL);
}

// Keys of the batched candidate blocks (all of them into `all`, count in
// cd.counters[4]) and of those without a device slot (new blocks, or blocks
// held by the host store) into `req`.
__global__ void stream_req_batch_kernel(CandDev cd, uint64_t* all, uint64_t* req, uint32_t* count, uint32_t cap)
{
    const uint32_t n = min(cd.counters[4], cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        all[i] = cd.skey[i];
        if (cd.sslot[i] >= 0) continue;
        const uint32_t p = atomicAdd(count, 1u);
        if (p < cap) req[p] = cd.skey[i];
    }
}

// The same for the plain path's candidate list (its length in
// counters[parity]).
__global__ void stream_req_plain_kernel(CandDev cd, VolDev v, int parity, uint64_t* all, uint64_t* req,
                                        uint32_t* count, uint32_t cap)
{
    const uint32_t n = min(min(cd.counters[parity], cd.cap), cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t key = cd.keys[cd.list[i]];
        all[i] = key;
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        if (vol_find(v, key, bx, by, bz) >= 0) continue;
        const uint32_t p = atomicAdd(count, 1u);
        if (p < cap) req[p] = key;
    }
}

// Streamed-in blocks i < n take pool slots base + i: data, key, hash entry.
__global__ void stream_in_kernel(VolDev v, const uint64_t* __restrict__ keys, const float* __restrict__ data,
                                 int64_t n, int64_t base)
{
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const int slot = (int)(base + i);
    float* dst = v.pool + (size_t)slot * v.stride;
    const float* src = data + (size_t)i * v.stride;
    for (int k = threadIdx.x; k < v.stride; k += blockDim.x) dst[k] = src[k];
    if (threadIdx.x == 0) {
        v.slot_keys[slot] = keys[i];
        hash_put(v, keys[i], slot);
    }
}

// Looks up the pool slot of every batched candidate again (blocks were
// streamed in, or moved by a compaction).
__global__ void sslot_refresh_kernel(CandDev cd, VolDev v)
{
    const uint32_t n = cd.counters[4];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int bx, by, bz;
        unpack_key(cd.skey[i], bx, by, bz);
        cd.sslot[i] = vol_find(v, cd.skey[i], bx, by, bz);
    }
}

// Copies the blocks of slots[i] into staging position i.
__global__ void stream_gather_kernel(VolDev v, const int32_t* __restrict__ slots, int64_t n, float* out)
{
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const float* src = v.pool + (size_t)slots[i] * v.stride;
    float* dst = out + (size_t)i * v.stride;
    for (int k = threadIdx.x; k < v.stride; k += blockDim.x) dst[k] = src[k];
}

// Moves block from[i] to slot to[i] (the two ranges are disjoint).
__global__ void stream_move_kernel(VolDev v, const int32_t* __restrict__ from, const int32_t* __restrict__ to,
                                   int64_t n)
{
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const float* src = v.pool + (size_t)from[i] * v.stride;
    float* dst = v.pool + (size_t)to[i] * v.stride;
    for (int k = threadIdx.x; k < v.stride; k += blockDim.x) dst[k] = src[k];
    if (threadIdx.x == 0) v.slot_keys[to[i]] = v.slot_keys[from[i]];
}

// Re-inserts the blocks of slots [0, n) into the (cleared) hash table.
__global__ void hash_rebuild_kernel(VolDev v, int64_t n)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
        hash_put(v, v.slot_keys[s], (int)s);
}

__global__ void set_count_kernel(uint32_t* p, uint32_t x) { *p = x; }

__global__ void set_error_kernel(int32_t* err, int32_t code) { set_error(err, code); }

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static bool grow_stage(StreamStore* st, size_t blocks)
{
    if (blocks <= st->stage_cap) return true;
    const size_t cap = std::max(blocks, 2 * st->stage_cap);
    if (hipDeviceSynchronize() != hipSuccess) return false;
    if (st->h_stage) (void)hipHostFree(st->h_stage);
    (void)hipFree(st->d_stage);
    st->h_stage = nullptr;
    st->d_stage = nullptr;
    st->stage_cap = 0;
    if (hipHostMalloc((void**)&st->h_stage, cap * st->block_bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&st->d_stage, cap * st->block_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    st->stage_cap = cap;
    return true;
}

static bool grow_keys(StreamStore* st, size_t n)
{
    if (n <= st->keys_cap) return true;
    const size_t cap = std::max(n, 2 * st->keys_cap);
    if (hipDeviceSynchronize() != hipSuccess) return false;
    if (st->h_keys) (void)hipHostFree(st->h_keys);
    if (st->h_slots) (void)hipHostFree(st->h_slots);
    (void)hipFree(st->d_keys);
    (void)hipFree(st->d_all);
    (void)hipFree(st->d_slots);
    st->h_keys = nullptr;
    st->h_slots = nullptr;
    st->d_keys = nullptr;
    st->d_all = nullptr;
    st->d_slots = nullptr;
    st->keys_cap = 0;
    if (hipHostMalloc((void**)&st->h_keys, cap * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&st->h_slots, 2 * cap * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&st->d_keys, cap * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&st->d_all, cap * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&st->d_slots, 2 * cap * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    st->keys_cap = cap;
    return true;
}

static size_t host_slot(StreamStore* st)
{
    if (!st->free_slots.empty()) {
        const size_t s = st->free_slots.back();
        st->free_slots.pop_back();
        return s;
    }
    const size_t s = st->n_slots++;
    st->arena.resize(st->n_slots * st->block_bytes);
    return s;
}

static bool streaming(const sc_volume* vol) { return vol->stream && vol->stream->enabled; }

int64_t stream_host_blocks(const sc_volume* vol) { return vol->stream ? (int64_t)vol->stream->where.size() : 0; }

static sc_status read_n_blocks(sc_volume* vol, hipStream_t s, int64_t& nb)
{
    int32_t err = 0;
    const sc_status st = sc_volume_query(vol, s, &nb, &err);
    if (st != SC_OK) return st;
    return err;
}

static sc_status d2h(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return SC_OK;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return SC_EDEVICE;
    return SC_OK;
}

// Keys of the device blocks, in slot order.
static sc_status device_keys(sc_volume* vol, hipStream_t s, std::vector<uint64_t>& keys)
{
    int64_t nb = 0;
    const sc_status e = read_n_blocks(vol, s, nb);
    if (e != SC_OK) return e;
    keys.resize((size_t)nb);
    return d2h(keys.data(), vol->dev.slot_keys, sizeof(uint64_t) * (size_t)nb, s);
}

// Streams in the host-held blocks among `want` (host keys), appending them
// to the pool.  Synchronises `s`.
static sc_status stream_in_keys(sc_volume* vol, const std::vector<uint64_t>& want, hipStream_t s, size_t& moved)
{
    StreamStore* st = vol->stream;
    moved = 0;
    std::vector<std::pair<uint64_t, size_t>> take;
    for (uint64_t k : want) {
        auto it = st->where.find(k);
        if (it != st->where.end()) take.emplace_back(it->first, it->second);
    }
    if (take.empty()) return SC_OK;
    int64_t nb = 0;
    sc_status e = read_n_blocks(vol, s, nb);
    if (e != SC_OK) return e;
    const size_t m = take.size();
    if (nb + (int64_t)m > vol->p.max_blocks) {
        // the work cannot run with every block it may touch: the field is
        // left unspecified, as for any full pool
        set_error_kernel<<<1, 1, 0, s>>>(vol->dev.err, SC_EPOOLFULL);
        return SC_EPOOLFULL;
    }
    if (!grow_stage(st, m) || !grow_keys(st, m)) return SC_ENOMEM;
    for (size_t i = 0; i < m; ++i) {
        memcpy(st->h_stage + i * st->block_bytes, st->arena.data() + take[i].second * st->block_bytes,
               st->block_bytes);
        st->h_keys[i] = take[i].first;
    }
    if (hipMemcpyAsync(st->d_stage, st->h_stage, m * st->block_bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(st->d_keys, st->h_keys, m * sizeof(uint64_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return SC_EDEVICE;
    stream_in_kernel<<<(unsigned)m, 256, 0, s>>>(vol->dev, st->d_keys, reinterpret_cast<const float*>(st->d_stage),
                                                 (int64_t)m, nb);
    set_count_kernel<<<1, 1, 0, s>>>(vol->dev.n_blocks, (uint32_t)(nb + (int64_t)m));
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SC_EDEVICE;
    for (const auto& kv : take) {
        st->free_slots.push_back(kv.second);
        st->where.erase(kv.first);
    }
    st->blocks_in += (int64_t)m;
    moved = m;
    return SC_OK;
}

// Moves the device blocks whose index `out` marks to the host store and
// compacts the pool: the live blocks above the new count fill the holes
// below it (disjoint ranges), the freed slots are cleared to the empty
// state, and the hash table is rebuilt.
static sc_status evict(sc_volume* vol, const std::vector<uint64_t>& keys, const std::vector<char>& out, hipStream_t s)
{
    StreamStore* st = vol->stream;
    const int64_t nb = (int64_t)keys.size();
    std::vector<int32_t> gone, holes, movers;
    for (int64_t i = 0; i < nb; ++i)
        if (out[i]) gone.push_back((int32_t)i);
    if (gone.empty()) return SC_OK;
    const int64_t live = nb - (int64_t)gone.size();
    for (int32_t g : gone)
        if (g < live) holes.push_back(g);
    for (int64_t i = live; i < nb; ++i)
        if (!out[i]) movers.push_back((int32_t)i);
    if (holes.size() != movers.size()) return SC_EDEVICE;
    const size_t e = gone.size();
    if (!grow_stage(st, e) || !grow_keys(st, std::max(e, movers.size()))) return SC_ENOMEM;
    // evicted blocks to the host
    memcpy(st->h_slots, gone.data(), e * sizeof(int32_t));
    if (hipMemcpyAsync(st->d_slots, st->h_slots, e * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return SC_EDEVICE;
    stream_gather_kernel<<<(unsigned)e, 256, 0, s>>>(vol->dev, st->d_slots, (int64_t)e,
                                                     reinterpret_cast<float*>(st->d_stage));
    sc_status r = d2h(st->h_stage, st->d_stage, e * st->block_bytes, s);
    if (r != SC_OK) return r;
    for (size_t i = 0; i < e; ++i) {
        const uint64_t key = keys[gone[i]];
        const size_t hs = host_slot(st);
        memcpy(st->arena.data() + hs * st->block_bytes, st->h_stage + i * st->block_bytes, st->block_bytes);
        st->where[key] = hs;
    }
    st->blocks_out += (int64_t)e;
    // compaction
    const size_t m = movers.size();
    if (m > 0) {
        memcpy(st->h_slots, movers.data(), m * sizeof(int32_t));
        memcpy(st->h_slots + m, holes.data(), m * sizeof(int32_t));
        if (hipMemcpyAsync(st->d_slots, st->h_slots, 2 * m * sizeof(int32_t), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return SC_EDEVICE;
        stream_move_kernel<<<(unsigned)m, 256, 0, s>>>(vol->dev, st->d_slots, st->d_slots + m, (int64_t)m);
    }
    fill_u64(vol->dev.keys, kKeyEmpty, (size_t)vol->p.n_buckets, s);
    fill_u32(reinterpret_cast<uint32_t*>(vol->dev.vals), 0xFFFFFFFFu, (size_t)vol->p.n_buckets, s);
    if (live > 0) hash_rebuild_kernel<<<vol->n_cu * 4, 256, 0, s>>>(vol->dev, live);
    set_count_kernel<<<1, 1, 0, s>>>(vol->dev.n_blocks, (uint32_t)live);
    fill_u32(reinterpret_cast<uint32_t*>(vol->dev.pool + (size_t)vol->dev.stride * live), 0u,
             (size_t)vol->dev.stride * (size_t)(nb - live), s);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SC_EDEVICE;
    return SC_OK;
}

// Before a voxel pass in streaming mode: the candidate keys of the work are
// in d_all (ncand of them) and those without a device slot in d_keys (their
// number in d_req).  When the pool cannot take all of the latter, resident
// blocks that are not candidates are streamed out, farthest from the
// candidates' mean first, until it can (with an eighth of the pool to
// spare when possible).  Then the host-held ones are streamed in.  `moved`
// tells whether any pool slot changed.
static sc_status prepare_work(sc_volume* vol, hipStream_t s, uint32_t ncand, bool& moved)
{
    StreamStore* st = vol->stream;
    moved = false;
    uint32_t n = 0;
    sc_status e = d2h(&n, st->d_req, sizeof(uint32_t), s);
    if (e != SC_OK) return e;
    if (n > st->keys_cap) return SC_ENOMEM;
    if (n == 0) return SC_OK;
    std::vector<uint64_t> want(n);
    e = d2h(want.data(), st->d_keys, sizeof(uint64_t) * n, s);
    if (e != SC_OK) return e;
    int64_t nb = 0;
    e = read_n_blocks(vol, s, nb);
    if (e != SC_OK) return e;
    const int64_t cap = vol->p.max_blocks;
    if (nb + (int64_t)n > cap) {
        std::vector<uint64_t> cand(ncand);
        e = d2h(cand.data(), st->d_all, sizeof(uint64_t) * ncand, s);
        if (e != SC_OK) return e;
        std::unordered_map<uint64_t, char> is_cand;
        is_cand.reserve(ncand * 2);
        double mx = 0.0, my = 0.0, mz = 0.0;
        for (uint64_t k : cand) {
            is_cand[k] = 1;
            int bx, by, bz;
            unpack_key(k, bx, by, bz);
            mx += bx;
            my += by;
            mz += bz;
        }
        if (ncand) {
            mx /= ncand;
            my /= ncand;
            mz /= ncand;
        }
        std::vector<uint64_t> keys;
        e = device_keys(vol, s, keys);
        if (e != SC_OK) return e;
        std::vector<std::pair<double, size_t>> far;
        for (size_t i = 0; i < keys.size(); ++i) {
            if (is_cand.count(keys[i])) continue;
            int bx, by, bz;
            unpack_key(keys[i], bx, by, bz);
            const double dx = bx - mx, dy = by - my, dz = bz - mz;
            far.emplace_back(-(dx * dx + dy * dy + dz * dz), i);
        }
        std::sort(far.begin(), far.end());
        // blocks that may stay: room for the requests, and an eighth of the
        // pool to spare when there is room for that too
        const int64_t room = cap - (int64_t)n;
        const int64_t keep = (room - cap / 8 >= 0) ? room - cap / 8 : room;
        const int64_t need = std::max<int64_t>(0, std::min<int64_t>((int64_t)keys.size() - keep, (int64_t)far.size()));
        std::vector<char> out(keys.size(), 0);
        for (int64_t i = 0; i < need; ++i) out[far[(size_t)i].second] = 1;
        e = evict(vol, keys, out, s);
        if (e != SC_OK) return e;
        moved = need > 0;
        e = read_n_blocks(vol, s, nb);
        if (e != SC_OK) return e;
        if (nb + (int64_t)n > cap) {
            set_error_kernel<<<1, 1, 0, s>>>(vol->dev.err, SC_EPOOLFULL);
            return SC_EPOOLFULL;
        }
    }
    size_t in = 0;
    e = stream_in_keys(vol, want, s, in);
    if (e != SC_OK) return e;
    moved = moved || in > 0;
    return SC_OK;
}

// A streaming step that failed after the candidates were generated leaves
// the operation undone and its candidate entries in place: the failure is
// made sticky, so the volume is reset before further use.
static sc_status fail_sticky(sc_volume* vol, sc_status e, hipStream_t s)
{
    if (e != SC_OK && e != SC_EPOOLFULL) set_error_kernel<<<1, 1, 0, s>>>(vol->dev.err, e);
    return e;
}

static sc_status stream_in_batch_impl(sc_volume* vol, hipStream_t s);
static sc_status stream_in_plain_impl(sc_volume* vol, int parity, hipStream_t s);

sc_status stream_in_batch(sc_volume* vol, hipStream_t s)
{
    return streaming(vol) ? fail_sticky(vol, stream_in_batch_impl(vol, s), s) : SC_OK;
}

sc_status stream_in_plain(sc_volume* vol, int parity, hipStream_t s)
{
    return streaming(vol) ? fail_sticky(vol, stream_in_plain_impl(vol, parity, s), s) : SC_OK;
}

// Batched path, after the candidate stage: room for every candidate block,
// the host-held ones streamed in, and the candidates' pool slots refreshed.
static sc_status stream_in_batch_impl(sc_volume* vol, hipStream_t s)
{
    StreamStore* st = vol->stream;
    if (!grow_keys(st, vol->cand_buckets)) return SC_ENOMEM;
    set_count_kernel<<<1, 1, 0, s>>>(st->d_req, 0u);
    stream_req_batch_kernel<<<vol->n_cu * 4, 256, 0, s>>>(vol->cand, st->d_all, st->d_keys, st->d_req,
                                                          (uint32_t)st->keys_cap);
    uint32_t ncand = 0;
    sc_status e = d2h(&ncand, vol->cand.counters + 4, sizeof(uint32_t), s);
    if (e != SC_OK) return e;
    bool moved = false;
    e = prepare_work(vol, s, std::min<uint32_t>(ncand, (uint32_t)st->keys_cap), moved);
    if (e != SC_OK) return e;
    if (moved) sslot_refresh_kernel<<<vol->n_cu * 4, 256, 0, s>>>(vol->cand, vol->dev);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

// Plain path, after the candidate list of one operation is built (the
// update kernel looks its blocks up itself).
static sc_status stream_in_plain_impl(sc_volume* vol, int parity, hipStream_t s)
{
    StreamStore* st = vol->stream;
    if (!grow_keys(st, vol->cand.cap)) return SC_ENOMEM;
    set_count_kernel<<<1, 1, 0, s>>>(st->d_req, 0u);
    stream_req_plain_kernel<<<vol->n_cu * 4, 256, 0, s>>>(vol->cand, vol->dev, parity, st->d_all, st->d_keys,
                                                          st->d_req, (uint32_t)st->keys_cap);
    uint32_t ncand = 0;
    sc_status e = d2h(&ncand, vol->cand.counters + parity, sizeof(uint32_t), s);
    if (e != SC_OK) return e;
    bool moved = false;
    return prepare_work(vol, s, std::min<uint32_t>(std::min<uint32_t>(ncand, vol->cand.cap), (uint32_t)st->keys_cap),
                        moved);
}

void stream_clear(sc_volume* vol)
{
    StreamStore* st = vol->stream;
    if (!st) return;
    st->where.clear();
    st->free_slots.clear();
    st->arena.clear();
    st->arena.shrink_to_fit();
    st->n_slots = 0;
}

void stream_destroy(sc_volume* vol)
{
    StreamStore* st = vol->stream;
    if (!st) return;
    if (st->h_stage) (void)hipHostFree(st->h_stage);
    if (st->h_keys) (void)hipHostFree(st->h_keys);
    if (st->h_slots) (void)hipHostFree(st->h_slots);
    (void)hipFree(st->d_stage);
    (void)hipFree(st->d_keys);
    (void)hipFree(st->d_all);
    (void)hipFree(st->d_slots);
    (void)hipFree(st->d_req);
    delete st;
    vol->stream = nullptr;
}

}  // namespace sc

using namespace sc;

extern "C" {

sc_status sc_stream_enable(sc_volume* vol, int32_t enable)
{
    if (!vol) return SC_EINVAL;
    if (!vol->stream) {
        vol->stream = new (std::nothrow) StreamStore();
        if (!vol->stream) return SC_ENOMEM;
        vol->stream->block_bytes = sizeof(float) * (size_t)vol->dev.stride;
        if (hipMalloc(&vol->stream->d_req, sizeof(uint32_t)) != hipSuccess) {
            stream_destroy(vol);
            return SC_ENOMEM;
        }
    }
    if (!enable && !vol->stream->where.empty()) return SC_EINVAL;  // blocks still on the host
    vol->stream->enabled = enable != 0;
    return SC_OK;
}

sc_status sc_stream_out(sc_volume* vol, const double* center, double radius, void* stream)
{
    if (!vol || !center || !(radius >= 0.0)) return SC_EINVAL;
    if (!streaming(vol)) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint64_t> keys;
    sc_status e = device_keys(vol, s, keys);
    if (e != SC_OK) return e;
    // block centre: voxel centres s * n for n in [8 b, 8 b + 7], so 8 b + 3.5
    const double vs = (double)vol->p.voxel_size, r2 = radius * radius;
    std::vector<char> out(keys.size(), 0);
    for (size_t i = 0; i < keys.size(); ++i) {
        int bx, by, bz;
        unpack_key(keys[i], bx, by, bz);
        const double dx = vs * (8.0 * bx + 3.5) - center[0];
        const double dy = vs * (8.0 * by + 3.5) - center[1];
        const double dz = vs * (8.0 * bz + 3.5) - center[2];
        out[i] = (dx * dx + dy * dy + dz * dz > r2) ? 1 : 0;
    }
    return evict(vol, keys, out, s);
}

sc_status sc_stream_in_all(sc_volume* vol, void* stream)
{
    if (!vol) return SC_EINVAL;
    if (!vol->stream || vol->stream->where.empty()) return SC_OK;
    std::vector<uint64_t> want;
    want.reserve(vol->stream->where.size());
    for (const auto& kv : vol->stream->where) want.push_back(kv.first);
    size_t in = 0;
    return stream_in_keys(vol, want, (hipStream_t)stream, in);
}

sc_status sc_stream_export(sc_volume* vol, int32_t* block_xyz, float* D, float* W, void* C, int64_t cap,
                           int64_t* n_out)
{
    if (!vol || cap < 0) return SC_EINVAL;
    const StreamStore* st = vol->stream;
    const int64_t n = st ? (int64_t)st->where.size() : 0;
    if (n_out) *n_out = n;
    if (!st) return SC_OK;
    const bool rgba = vol->p.color_mode == SC_COLOR_RGBA8;
    int64_t b = 0;
    for (const auto& kv : st->where) {
        if (b >= cap) break;
        const float* rec = reinterpret_cast<const float*>(st->arena.data() + kv.second * st->block_bytes);
        int x, y, z;
        unpack_key(kv.first, x, y, z);
        if (block_xyz) {
            block_xyz[3 * b] = x;
            block_xyz[3 * b + 1] = y;
            block_xyz[3 * b + 2] = z;
        }
        const double* Dd = reinterpret_cast<const double*>(rec);
        for (int i = 0; i < kBlockVox; ++i) {
            if (D) D[b * kBlockVox + i] = (float)Dd[i];
            if (W) W[b * kBlockVox + i] = rec[kPoolW + i];
        }
        if (C) {
            if (rgba) {
                memcpy(reinterpret_cast<uint32_t*>(C) + b * kBlockVox, rec + kPoolC, sizeof(uint32_t) * kBlockVox);
            } else {
                const double* Cd = reinterpret_cast<const double*>(rec + kPoolC);
                float* Cf = reinterpret_cast<float*>(C) + b * 3 * kBlockVox;
                for (int i = 0; i < 3 * kBlockVox; ++i) Cf[i] = (float)Cd[i];
            }
        }
        ++b;
    }
    return SC_OK;
}

sc_status sc_stream_stats(sc_volume* vol, void* stream, int64_t* stats)
{
    if (!vol || !stats) return SC_EINVAL;
    int64_t nb = 0;
    const sc_status e = sc_volume_query(vol, stream, &nb, nullptr);
    if (e != SC_OK) return e;
    const StreamStore* st = vol->stream;
    const int64_t bb = (int64_t)sizeof(float) * vol->dev.stride;
    stats[0] = nb;
    stats[1] = st ? (int64_t)st->where.size() : 0;
    stats[2] = st ? st->blocks_out : 0;
    stats[3] = st ? st->blocks_in : 0;
    stats[4] = st ? st->blocks_out * bb : 0;
    stats[5] = st ? st->blocks_in * bb : 0;
    return SC_OK;
}

}  // extern "C"
