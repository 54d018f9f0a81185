// Iso-surface extraction (Sec. 3 "SDF volume": Marching Cubes over the SDF)
// and the surface metrics of Sec. 5 (mean absolute deviation of
// nearest-neighbour distances between point sets: CORR and COMPL).
#include <string.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "internal.hpp"
#include "kernels.hpp"

#define MESH_TRY(x)                               \
    do {                                          \
        if ((x) != hipSuccess) return SC_EDEVICE; \
    } while (0)

namespace sc {

// ---------------------------------------------------------------------------
// case table
// ---------------------------------------------------------------------------

// Corner k of the cube of voxel n sits at n + (k & 1, (k >> 1) & 1, k >> 2).
// Edge e = 4 a + o1 + 2 o2 runs along axis a from the corner whose offsets on
// the two other axes (in increasing axis order) are (o1, o2).  A corner is
// inside when D < 0.  The table is built on the host from a rule: on each
// face, with its corners counter-clockwise about the outward normal, every
// run of inside corners is cut off by a segment from the edge that enters
// the run to the edge that leaves it (diagonal inside corners of a face stay
// apart, identically on both cubes sharing the face).  Segments chain across
// faces into loops; loops are ordered by their smallest edge and start
// there.  A loop holding two segments of one face is fanned around an added
// centre vertex (the mean of its vertices, summed in loop order), any other
// loop from its first vertex, so no triangle side lies inside a face.
//
// Per case, 16 bytes: loops in order, each a header byte (length, | 0x80
// when fanned around a centre) followed by its edges; a zero header (or the
// end of the 16 bytes) ends the case.
struct McTable {
    uint8_t loops[256][16];
    uint8_t ntri[256];
};

static __device__ McTable g_mc;

static int mc_corner(const int off[3]) { return off[0] + 2 * off[1] + 4 * off[2]; }

static int mc_edge_between(int k0, int k1)
{
    const int o0[3] = {k0 & 1, (k0 >> 1) & 1, (k0 >> 2) & 1};
    const int o1[3] = {k1 & 1, (k1 >> 1) & 1, (k1 >> 2) & 1};
    int a = 0;
    while (o0[a] == o1[a]) ++a;
    const int* lo = (o0[a] < o1[a]) ? o0 : o1;
    int other[2], m = 0;
    for (int b = 0; b < 3; ++b)
        if (b != a) other[m++] = b;
    return 4 * a + lo[other[0]] + 2 * lo[other[1]];
}

static bool mc_build(McTable& T)
{
    memset(&T, 0, sizeof(T));
    int ring[6][4];
    for (int a = 0; a < 3; ++a) {
        const int u = (a + 1) % 3, v = (a + 2) % 3;
        static const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};  // counter-clockwise about +e_a
        for (int side = 0; side < 2; ++side) {
            for (int i = 0; i < 4; ++i) {
                int off[3];
                off[a] = side;
                off[u] = uv[i][0];
                off[v] = uv[i][1];
                // about -e_a on the low face: the same corners in reverse
                ring[2 * a + side][side ? i : 3 - i] = mc_corner(off);
            }
        }
    }
    for (int c = 0; c < 256; ++c) {
        int next[12], face[12];
        for (int e = 0; e < 12; ++e) next[e] = face[e] = -1;
        for (int f = 0; f < 6; ++f) {
            int ce[4], enters[4], n = 0;
            for (int i = 0; i < 4; ++i) {
                const int k0 = ring[f][i], k1 = ring[f][(i + 1) & 3];
                const int in0 = (c >> k0) & 1, in1 = (c >> k1) & 1;
                if (in0 != in1) {
                    ce[n] = mc_edge_between(k0, k1);
                    enters[n] = in1;
                    ++n;
                }
            }
            for (int j = 0; j < n; ++j)
                if (enters[j]) {
                    next[ce[j]] = ce[(j + 1) % n];
                    face[ce[j]] = f;
                }
        }
        bool seen[12] = {};
        int p = 0, ntri = 0;
        for (int e0 = 0; e0 < 12; ++e0) {
            if (next[e0] < 0 || seen[e0]) continue;
            uint8_t loop[12];
            int len = 0, e = e0;
            unsigned fmask = 0;
            bool centre = false;
            while (!seen[e]) {
                seen[e] = true;
                loop[len++] = (uint8_t)e;
                centre |= ((fmask >> face[e]) & 1u) != 0;
                fmask |= 1u << face[e];
                e = next[e];
            }
            if (p + 1 + len > 16) return false;  // at most four loops over twelve edges: never
            T.loops[c][p++] = (uint8_t)(len | (centre ? 0x80 : 0));
            for (int i = 0; i < len; ++i) T.loops[c][p++] = loop[i];
            ntri += centre ? len : len - 2;
        }
        T.ntri[c] = (uint8_t)ntri;
    }
    return true;
}

static sc_status mc_table_ready()
{
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    MESH_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return SC_EDEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!done[dev]) {
        McTable T;
        if (!mc_build(T)) return SC_EDEVICE;
        MESH_TRY(hipMemcpyToSymbol(HIP_SYMBOL(g_mc), &T, sizeof(T), 0, hipMemcpyHostToDevice));
        done[dev] = true;
    }
    return SC_OK;
}

// ---------------------------------------------------------------------------
// Marching Cubes: one wavefront per allocated block; the block and its +x,
// +y, +z neighbours' first layers (9 x 9 x 9 voxels) are staged in LDS and
// each lane meshes eight cubes.  A count pass stores each block's triangle
// count, a scan turns the counts into offsets, and the fill pass writes each
// block's triangles from its offset: no shared counter, and the output order
// is fixed (pool order, then cube order).
// ---------------------------------------------------------------------------

struct MeshOut {
    float* xyz;                  // cap x 3 x 3, or null
    int32_t* keys;               // cap x 3 x 4, or null
    uint32_t* counts;            // count pass: triangles per block (else null)
    const uint64_t* offsets;     // fill pass: first triangle of each block
    int64_t cap;
};

// Position (FP64, metres) and key (x, y, z, axis) of the vertex on edge e of
// the cube whose corner 0 is LDS cell r0 and voxel g.
__device__ inline void mc_edge_vertex(int e, const double* sD, int r0, const int g[3], double s, double p[3],
                                      int key[4])
{
    const int a = e >> 2, r = e & 3;
    const int o1 = (a == 0) ? 1 : 0, o2 = (a == 2) ? 1 : 2;
    int off[3] = {0, 0, 0};
    off[o1] = r & 1;
    off[o2] = r >> 1;
    const int lo = r0 + off[0] + 9 * off[1] + 81 * off[2];
    const int hi = lo + ((a == 0) ? 1 : (a == 1) ? 9 : 81);
    const double d0 = sD[lo], d1 = sD[hi];
    const double t = d0 / (d0 - d1);
    const int q[3] = {g[0] + off[0], g[1] + off[1], g[2] + off[2]};
#pragma unroll
    for (int b = 0; b < 3; ++b) p[b] = s * (double)q[b];
    p[a] = s * ((double)q[a] + t);
    key[0] = q[0];
    key[1] = q[1];
    key[2] = q[2];
    key[3] = a;
}

__device__ inline void mc_put(const MeshOut& out, unsigned long long t, int corner, const double p[3], const int key[4])
{
    if (out.xyz) {
        float* o = out.xyz + (t * 3 + corner) * 3;
        o[0] = (float)p[0];
        o[1] = (float)p[1];
        o[2] = (float)p[2];
    }
    if (out.keys) {
        int32_t* k = out.keys + (t * 3 + corner) * 4;
        k[0] = key[0];
        k[1] = key[1];
        k[2] = key[2];
        k[3] = key[3];
    }
}

__global__ __launch_bounds__(64) void mesh_kernel(VolDev v, MeshOut out)
{
    __shared__ double sD[729];
    __shared__ float sW[729];
    __shared__ int nslot[8];
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    int bx, by, bz;
    unpack_key(v.slot_keys[b], bx, by, bz);
    if (lane < 8) {
        const int x = bx + (lane & 1), y = by + ((lane >> 1) & 1), z = bz + (lane >> 2);
        nslot[lane] = (lane == 0) ? b : vol_find(v, pack_key(x, y, z), x, y, z);
    }
    __syncthreads();
    for (int i = lane; i < 729; i += 64) {
        const int x = i % 9, y = (i / 9) % 9, z = i / 81;
        const int slot = nslot[(x >> 3) | ((y >> 3) << 1) | ((z >> 3) << 2)];
        const int li = (x & 7) + 8 * (y & 7) + 64 * (z & 7);
        double d = 0.0;
        float w = 0.0f;
        if (slot >= 0) {
            const float* blk = v.pool + (size_t)slot * v.stride;
            d = reinterpret_cast<const double*>(blk)[li];
            w = blk[kPoolW + li];
        }
        sD[i] = d;
        sW[i] = w;
    }
    __syncthreads();
    uint32_t cases[8];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int c = lane + 64 * j;
        const int r0 = (c & 7) + 9 * ((c >> 3) & 7) + 81 * (c >> 6);
        bool ok = true;
        uint32_t cs = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = r0 + (k & 1) + 9 * ((k >> 1) & 1) + 81 * (k >> 2);
            ok &= sW[r] > 0.0f;
            cs |= (sD[r] < 0.0 ? 1u : 0u) << k;
        }
        cases[j] = ok ? cs : 0u;
        mine += g_mc.ntri[cases[j]];
    }
    // wavefront-exclusive prefix of the triangle counts: the count pass
    // stores the block's total, the fill pass writes from the block's offset
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (out.counts) {
        if (lane == 63) out.counts[b] = incl;
        return;
    }
    unsigned long long t = out.offsets[b] + (incl - mine);
    const double s = (double)v.s;
    for (int j = 0; j < 8; ++j) {
        const uint32_t cs = cases[j];
        if (g_mc.ntri[cs] == 0) continue;
        const int c = lane + 64 * j;
        const int r0 = (c & 7) + 9 * ((c >> 3) & 7) + 81 * (c >> 6);
        const int g[3] = {8 * bx + (c & 7), 8 * by + ((c >> 3) & 7), 8 * bz + (c >> 6)};
        const uint8_t* tab = g_mc.loops[cs];
        int p = 0, li = 0;
        while (p < 16 && tab[p]) {
            const int len = tab[p] & 0x7f;
            const bool centre = (tab[p] & 0x80) != 0;
            const uint8_t* L = tab + p + 1;
            double pc[3] = {0.0, 0.0, 0.0};
            int kc[4] = {g[0], g[1], g[2], 3 + li};
            if (centre) {
                for (int i = 0; i < len; ++i) {
                    double q[3];
                    int kq[4];
                    mc_edge_vertex(L[i], sD, r0, g, s, q, kq);
                    pc[0] = pc[0] + q[0];
                    pc[1] = pc[1] + q[1];
                    pc[2] = pc[2] + q[2];
                }
                pc[0] = pc[0] / (double)len;
                pc[1] = pc[1] / (double)len;
                pc[2] = pc[2] / (double)len;
            }
            const int n_t = centre ? len : len - 2;
            for (int i = 0; i < n_t; ++i, ++t) {
                if (t >= (unsigned long long)out.cap) continue;
                double q[3];
                int kq[4];
                if (centre) {
                    mc_put(out, t, 0, pc, kc);
                    mc_edge_vertex(L[i], sD, r0, g, s, q, kq);
                    mc_put(out, t, 1, q, kq);
                    mc_edge_vertex(L[(i + 1) % len], sD, r0, g, s, q, kq);
                    mc_put(out, t, 2, q, kq);
                } else {
                    mc_edge_vertex(L[0], sD, r0, g, s, q, kq);
                    mc_put(out, t, 0, q, kq);
                    mc_edge_vertex(L[i + 1], sD, r0, g, s, q, kq);
                    mc_put(out, t, 1, q, kq);
                    mc_edge_vertex(L[i + 2], sD, r0, g, s, q, kq);
                    mc_put(out, t, 2, q, kq);
                }
            }
            p += 1 + len;
            ++li;
        }
    }
}

// Exclusive scan of per-block triangle counts into 64-bit offsets: 1024
// counts per workgroup, then one workgroup scans the workgroup sums in
// chunks with a running carry, then the carries are added.
__global__ __launch_bounds__(256) void scan_local_kernel(const uint32_t* __restrict__ in, uint64_t* out, uint64_t* sums,
                                                         uint32_t n)
{
    __shared__ uint64_t part[256];
    const uint32_t i0 = (blockIdx.x * 256u + threadIdx.x) * 4u;
    uint64_t v[4], mine = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (i0 + k < n) ? (uint64_t)in[i0 + k] : 0ull;
        mine += v[k];
    }
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint64_t y = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : 0ull;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = part[threadIdx.x] - mine;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < n) out[i0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

__global__ __launch_bounds__(256) void scan_sums_kernel(uint64_t* sums, uint32_t n, uint64_t* total)
{
    __shared__ uint64_t part[256];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0ull;
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n; c0 += 256u) {
        const uint32_t i = c0 + threadIdx.x;
        const uint64_t mine = (i < n) ? sums[i] : 0ull;
        part[threadIdx.x] = mine;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const uint64_t y = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : 0ull;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < n) sums[i] = carry + part[threadIdx.x] - mine;
        __syncthreads();
        if (threadIdx.x == 255) carry += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void scan_add_kernel(uint64_t* out, const uint64_t* __restrict__ sums, uint32_t n)
{
    const uint32_t i0 = (blockIdx.x * 256u + threadIdx.x) * 4u;
    const uint64_t c = sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n) out[i0 + k] += c;
}

// ---------------------------------------------------------------------------
// unique vertices: a hash set over vertex keys
// ---------------------------------------------------------------------------

constexpr int kKeyRange = 1 << 19;  // |voxel coordinate| bound of the vertex key packing

__device__ inline uint64_t vertex_key(const int32_t* k, bool& bad)
{
    bad |= k[0] < -kKeyRange || k[0] >= kKeyRange || k[1] < -kKeyRange || k[1] >= kKeyRange || k[2] < -kKeyRange ||
           k[2] >= kKeyRange || k[3] < 0 || k[3] > 7;
    return ((uint64_t)(k[0] & 0xFFFFF) << 43) | ((uint64_t)(k[1] & 0xFFFFF) << 23) | ((uint64_t)(k[2] & 0xFFFFF) << 3) |
           (uint64_t)(k[3] & 7);
}

constexpr int kVertPerThread = 8;  // vertex instances per thread: one reservation per 2048

// Inserts each vertex key into the hash set; the threads that insert a key
// first append its position.  A workgroup scans its winners in LDS and
// reserves their range with one atomic.
__global__ __launch_bounds__(256) void unique_vertex_kernel(const float* __restrict__ xyz, const int32_t* __restrict__ keys,
                                                            int64_t n, uint64_t* table, uint32_t mask, float* out,
                                                            int64_t cap, unsigned long long* count, int* err)
{
    __shared__ uint32_t part[256];
    __shared__ unsigned long long base;
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kVertPerThread;
    uint32_t won = 0u;
    bool bad = false;
    for (int k = 0; k < kVertPerThread; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        const uint64_t key = vertex_key(keys + 4 * i, bad);
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
        for (uint32_t probe = 0; probe <= mask; ++probe) {
            const uint64_t old = atomicCAS((unsigned long long*)(table + h), (unsigned long long)kKeyEmpty,
                                           (unsigned long long)key);
            if (old == kKeyEmpty) {
                won |= 1u << k;
                break;
            }
            if (old == key) break;
            h = (h + 1) & mask;
        }
    }
    const uint32_t mine = (uint32_t)__popc(won);
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t y = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    if (threadIdx.x == 255) base = atomicAdd(count, (unsigned long long)part[255]);
    __syncthreads();
    unsigned long long pos = base + part[threadIdx.x] - mine;
    for (int k = 0; k < kVertPerThread; ++k) {
        if (!((won >> k) & 1u)) continue;
        const int64_t i = i0 + k;
        if ((int64_t)pos < cap) {
            out[3 * pos] = xyz[3 * i];
            out[3 * pos + 1] = xyz[3 * i + 1];
            out[3 * pos + 2] = xyz[3 * i + 2];
        }
        ++pos;
    }
    if (bad) atomicOr(err, 1);
}

// ---------------------------------------------------------------------------
// capped nearest-neighbour distances over a uniform grid of cells of edge
// radius (1 + 2^-6): a point within the radius of a query lies in one of the
// 27 cells around the query's cell (the margin absorbs the rounding of the
// FP32 cell coordinate while |x| / radius stays below about 10^5)
// ---------------------------------------------------------------------------

struct NnGrid {
    uint64_t* keys;   // cell key per slot (kKeyEmpty = free)
    uint32_t* cnt;    // points per slot
    uint32_t* off;    // first point of each slot in `pts`
    uint32_t* cur;    // scatter cursor per slot
    float* pts;       // reference points sorted by slot (x, y, z)
    uint32_t mask;
    float inv;        // 1 / cell edge
};

__device__ inline int nn_cell(float x, float inv)
{
    const float c = floorf(x * inv);
    return (int)fminf(fmaxf(c, -1.0e6f), 1.0e6f);
}

__device__ inline int nn_find(const NnGrid& g, int cx, int cy, int cz)
{
    const uint64_t key = pack_key(cx, cy, cz);
    uint32_t h = hash_block(cx, cy, cz) & g.mask;
    for (uint32_t probe = 0; probe <= g.mask; ++probe) {
        const uint64_t k = g.keys[h];
        if (k == key) return (int)h;
        if (k == kKeyEmpty) return -1;
        h = (h + 1) & g.mask;
    }
    return -1;
}

__global__ __launch_bounds__(256) void nn_count_kernel(const float* __restrict__ ref, int64_t n, NnGrid g,
                                                       uint32_t* slot_of)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cx = nn_cell(ref[3 * i], g.inv), cy = nn_cell(ref[3 * i + 1], g.inv), cz = nn_cell(ref[3 * i + 2], g.inv);
    const uint64_t key = pack_key(cx, cy, cz);
    uint32_t h = hash_block(cx, cy, cz) & g.mask;
    for (uint32_t probe = 0; probe <= g.mask; ++probe) {
        const uint64_t old =
            atomicCAS((unsigned long long*)(g.keys + h), (unsigned long long)kKeyEmpty, (unsigned long long)key);
        if (old == kKeyEmpty || old == key) break;
        h = (h + 1) & g.mask;
    }
    slot_of[i] = h;
    atomicAdd(g.cnt + h, 1u);
}

constexpr int kSlotsPerThread = 16;  // grid slots per thread: one reservation per 4096

// Offsets: a workgroup scans its 4096 slots and reserves their range with one
// atomic (ranges of different workgroups need not be in slot order).
__global__ __launch_bounds__(256) void nn_offset_kernel(NnGrid g, uint32_t n_slots, uint32_t* total)
{
    __shared__ uint32_t part[256];
    __shared__ uint32_t base;
    const uint32_t i0 = (blockIdx.x * 256u + threadIdx.x) * kSlotsPerThread;
    uint32_t mine = 0u;
    for (int k = 0; k < kSlotsPerThread; ++k)
        if (i0 + k < n_slots) mine += g.cnt[i0 + k];
    part[threadIdx.x] = mine;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t y = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    if (threadIdx.x == 255) base = atomicAdd(total, part[255]);
    __syncthreads();
    uint32_t off = base + part[threadIdx.x] - mine;
    for (int k = 0; k < kSlotsPerThread; ++k)
        if (i0 + k < n_slots) {
            g.off[i0 + k] = off;
            off += g.cnt[i0 + k];
        }
}

__global__ __launch_bounds__(256) void nn_scatter_kernel(const float* __restrict__ ref, int64_t n, NnGrid g,
                                                         const uint32_t* __restrict__ slot_of)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t h = slot_of[i];
    const uint32_t pos = g.off[h] + atomicAdd(g.cur + h, 1u);
    g.pts[3 * (size_t)pos] = ref[3 * i];
    g.pts[3 * (size_t)pos + 1] = ref[3 * i + 1];
    g.pts[3 * (size_t)pos + 2] = ref[3 * i + 2];
}

__global__ __launch_bounds__(256) void nn_query_kernel(const float* __restrict__ q, int64_t n, NnGrid g, bool empty,
                                                       float radius, float* dist, double* sum)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mine = 0.0;
    if (i < n) {
        const float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
        float best = __builtin_inff();
        if (!empty) {
            const int cx = nn_cell(x, g.inv), cy = nn_cell(y, g.inv), cz = nn_cell(z, g.inv);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int h = nn_find(g, cx + dx, cy + dy, cz + dz);
                        if (h < 0) continue;
                        const uint32_t a = g.off[h], e = a + g.cnt[h];
                        for (uint32_t k = a; k < e; ++k) {
                            const float ex = x - g.pts[3 * (size_t)k];
                            const float ey = y - g.pts[3 * (size_t)k + 1];
                            const float ez = z - g.pts[3 * (size_t)k + 2];
                            best = fminf(best, (ex * ex + ey * ey) + ez * ez);
                        }
                    }
        }
        const float d = fminf(sqrtf(best), radius);
        if (dist) dist[i] = d;
        mine = (double)d;
    }
    if (sum) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
        if ((threadIdx.x & 63) == 0 && i - (threadIdx.x & 63) < n) atomicAdd(sum, mine);  // not a loop
    }
}

static uint32_t pow2_at_least(uint64_t x)
{
    uint32_t p = 1024;
    while (p < x && p < (1u << 30)) p <<= 1;
    return p;
}

}  // namespace sc

using namespace sc;

extern "C" {

sc_status sc_mesh_table(uint8_t* loops, uint8_t* ntri)
{
    if (!loops && !ntri) return SC_EINVAL;
    McTable T;
    if (!mc_build(T)) return SC_EDEVICE;
    if (loops) memcpy(loops, T.loops, sizeof(T.loops));
    if (ntri) memcpy(ntri, T.ntri, sizeof(T.ntri));
    return SC_OK;
}

sc_status sc_volume_mesh(sc_volume* vol, void* stream, float* tri_xyz, int32_t* tri_keys, int64_t cap, int64_t* n_tri)
{
    if (!vol || cap < 0 || !n_tri) return SC_EINVAL;
    sc_status st = mc_table_ready();
    if (st != SC_OK) return st;
    int64_t nb = 0;
    st = sc_volume_query(vol, stream, &nb, nullptr);
    if (st != SC_OK) return st;
    *n_tri = 0;
    if (nb == 0) return SC_OK;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t n = (uint32_t)nb;
    const uint32_t wgs = (n + 1023u) / 1024u;
    uint32_t* counts = nullptr;
    uint64_t *offsets = nullptr, *sums = nullptr, *d_total = nullptr;
    bool ok = hipMalloc(&counts, sizeof(uint32_t) * n) == hipSuccess;
    ok = ok && hipMalloc(&offsets, sizeof(uint64_t) * n) == hipSuccess;
    ok = ok && hipMalloc(&sums, sizeof(uint64_t) * wgs) == hipSuccess;
    ok = ok && hipMalloc(&d_total, sizeof(uint64_t)) == hipSuccess;
    const bool allocated = ok;
    uint64_t total = 0;
    if (ok) {
        MeshOut cnt{nullptr, nullptr, counts, nullptr, 0};
        mesh_kernel<<<n, 64, 0, s>>>(vol->dev, cnt);
        scan_local_kernel<<<wgs, 256, 0, s>>>(counts, offsets, sums, n);
        scan_sums_kernel<<<1, 256, 0, s>>>(sums, wgs, d_total);
        scan_add_kernel<<<wgs, 256, 0, s>>>(offsets, sums, n);
        if (cap > 0 && (tri_xyz || tri_keys)) {
            MeshOut fill{tri_xyz, tri_keys, nullptr, offsets, cap};
            mesh_kernel<<<n, 64, 0, s>>>(vol->dev, fill);
        }
        ok = hipGetLastError() == hipSuccess;
        ok = ok && hipMemcpyAsync(&total, d_total, sizeof(total), hipMemcpyDeviceToHost, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
    }
    (void)hipFree(counts);
    (void)hipFree(offsets);
    (void)hipFree(sums);
    (void)hipFree(d_total);
    if (!ok) return allocated ? SC_EDEVICE : SC_ENOMEM;
    *n_tri = (int64_t)total;
    return SC_OK;
}

sc_status sc_mesh_vertices(const float* tri_xyz, const int32_t* tri_keys, int64_t n_tri, float* vert_xyz, int64_t cap,
                           int64_t* n_vert, void* stream)
{
    if (n_tri < 0 || cap < 0 || !n_vert || (n_tri > 0 && (!tri_xyz || !tri_keys)) || (cap > 0 && !vert_xyz) ||
        n_tri > ((int64_t)1 << 28))
        return SC_EINVAL;
    *n_vert = 0;
    if (n_tri == 0) return SC_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nv = 3 * n_tri;
    const uint32_t slots = pow2_at_least((uint64_t)(2 * nv));
    uint64_t* table = nullptr;
    unsigned long long* d_count = nullptr;
    int* d_err = nullptr;
    bool ok = hipMalloc(&table, sizeof(uint64_t) * slots) == hipSuccess;
    ok = ok && hipMalloc(&d_count, sizeof(unsigned long long)) == hipSuccess;
    ok = ok && hipMalloc(&d_err, sizeof(int)) == hipSuccess;
    const bool allocated = ok;
    unsigned long long count = 0;
    int err = 0;
    if (ok) {
        fill_u64(table, kKeyEmpty, slots, s);
        ok = hipMemsetAsync(d_count, 0, sizeof(unsigned long long), s) == hipSuccess &&
             hipMemsetAsync(d_err, 0, sizeof(int), s) == hipSuccess;
        const int64_t per_wg = 256 * kVertPerThread;
        if (ok)
            unique_vertex_kernel<<<(unsigned)((nv + per_wg - 1) / per_wg), 256, 0, s>>>(
                tri_xyz, tri_keys, nv, table, slots - 1, vert_xyz, cap, d_count, d_err);
        ok = ok && hipGetLastError() == hipSuccess;
        ok = ok && hipMemcpyAsync(&count, d_count, sizeof(count), hipMemcpyDeviceToHost, s) == hipSuccess;
        ok = ok && hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess;
        ok = ok && hipStreamSynchronize(s) == hipSuccess;
    }
    (void)hipFree(table);
    (void)hipFree(d_count);
    (void)hipFree(d_err);
    if (!ok) return allocated ? SC_EDEVICE : SC_ENOMEM;
    if (err) return SC_ERANGE;
    *n_vert = (int64_t)count;
    return SC_OK;
}

sc_status sc_nn_distance(const float* ref, int64_t n_ref, const float* query, int64_t n_query, float radius,
                         float* dist, double* sum, void* stream)
{
    if (n_ref < 0 || n_query < 0 || (n_ref > 0 && !ref) || (n_query > 0 && !query) || !(radius > 0.0f) ||
        !(radius < 1.0e30f) || n_ref > ((int64_t)1 << 29) || n_query > ((int64_t)1 << 31))
        return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (sum && hipMemsetAsync(sum, 0, sizeof(double), s) != hipSuccess) return SC_EDEVICE;
    if (n_query == 0) return hipStreamSynchronize(s) == hipSuccess ? SC_OK : SC_EDEVICE;
    NnGrid g{};
    g.inv = 1.0f / (radius * (1.0f + 1.0f / 64.0f));
    const uint32_t slots = pow2_at_least((uint64_t)(2 * std::max<int64_t>(n_ref, 1)));
    g.mask = slots - 1;
    uint32_t* slot_of = nullptr;
    uint32_t* total = nullptr;
    bool ok = true, allocated = true;
    if (n_ref > 0) {
        ok = ok && hipMalloc(&g.keys, sizeof(uint64_t) * slots) == hipSuccess;
        ok = ok && hipMalloc(&g.cnt, sizeof(uint32_t) * slots) == hipSuccess;
        ok = ok && hipMalloc(&g.off, sizeof(uint32_t) * slots) == hipSuccess;
        ok = ok && hipMalloc(&g.cur, sizeof(uint32_t) * slots) == hipSuccess;
        ok = ok && hipMalloc(&g.pts, sizeof(float) * 3 * (size_t)n_ref) == hipSuccess;
        ok = ok && hipMalloc(&slot_of, sizeof(uint32_t) * (size_t)n_ref) == hipSuccess;
        ok = ok && hipMalloc(&total, sizeof(uint32_t)) == hipSuccess;
        allocated = ok;
        if (ok) {
            fill_u64(g.keys, kKeyEmpty, slots, s);
            fill_u32(g.cnt, 0u, slots, s);
            fill_u32(g.cur, 0u, slots, s);
            fill_u32(total, 0u, 1, s);
            const unsigned grid_r = (unsigned)((n_ref + 255) / 256);
            nn_count_kernel<<<grid_r, 256, 0, s>>>(ref, n_ref, g, slot_of);
            nn_offset_kernel<<<(slots + 256 * kSlotsPerThread - 1) / (256 * kSlotsPerThread), 256, 0, s>>>(g, slots,
                                                                                                          total);
            nn_scatter_kernel<<<grid_r, 256, 0, s>>>(ref, n_ref, g, slot_of);
        }
    }
    if (ok)
        nn_query_kernel<<<(unsigned)((n_query + 255) / 256), 256, 0, s>>>(query, n_query, g, n_ref == 0, radius, dist,
                                                                          sum);
    ok = ok && hipGetLastError() == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    (void)hipFree(g.keys);
    (void)hipFree(g.cnt);
    (void)hipFree(g.off);
    (void)hipFree(g.cur);
    (void)hipFree(g.pts);
    (void)hipFree(slot_of);
    (void)hipFree(total);
    return ok ? SC_OK : (allocated ? SC_EDEVICE : SC_ENOMEM);
}

}  // extern "C"
