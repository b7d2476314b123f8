// vm_ccl.hip -- connected-component labelling of the occupied voxels and the
// grouping of voxels into clusters (Sec. III-C, "Clustering", Alg. 1).
//
// Alg. 1 propagates the smaller label over every adjacency until nothing
// changes; from L_i = i its fixed point is the smallest index of each
// connected component.  That fixed point is reached here with a lock-free
// union-find over the occupied ranks (rank order == key order, so the
// smallest rank of a component is its smallest key):
//   * init:    every voxel points at the start of its run along x (runs of
//              consecutive occupied cells share a component trivially);
//   * merge:   runs in the four neighbouring rows with smaller keys
//              (dz = -1, any dy; dz = 0, dy = -1) are hooked together; a
//              voxel only hooks where an overlap between its run and a run of
//              the other row begins, plus the diagonal end cells, so each
//              pair of touching runs is hooked about once;
//   * flatten: every voxel takes its root.
// Hooks always put the larger root under the smaller one with a CAS on the
// root, so every root ends as the minimum of its tree and the labels are
// exact whatever the interleaving.  Path halving keeps trees shallow.  The
// 26-neighbourhood never needs the hash: occupancy and ranks come from the
// 1-bit-per-cell index.
#include "vm_common.h"
#include "vm_tilescan.h"

namespace vm {
namespace {

// Parent pointers are read through the ordinary caches.  A stale value is
// still an ancestor (parents only ever move to smaller ranks of the same
// component), so finds stay correct; the hook itself is a device-coherent
// CAS.  The path-halving and flattening stores are device-scope stores
// (written through to memory): with stores left in an XCD's L2, repeated
// labelling of one large map (5.3M voxels, 99k components) now and then left
// a voxel pointing at an intermediate ancestor after the flatten (3 calls in
// 400); with device-scope stores none did in 800.  Relaxed atomics keep the
// compiler from caching or tearing the accesses.
__device__ __forceinline__ uint32_t ld_parent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ void st_parent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool occ(const uint32_t* __restrict__ bits, uint32_t key)
{
    return (bits[key >> 5] >> (key & 31)) & 1u;
}

__device__ __forceinline__ uint32_t rank_of(const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wrank,
                                            uint32_t key)
{
    const uint32_t b = key & 31;
    return wrank[key >> 5] + __popc(bits[key >> 5] & ((1u << b) - 1u));
}

// Root of x with path halving (each visited node is re-pointed at its
// grandparent; concurrent writes only ever store an ancestor).
__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x)
{
    uint32_t p = ld_parent(&parent[x]);
    while (p != x) {
        const uint32_t g = ld_parent(&parent[p]);
        if (g == p) return p;
        st_parent(&parent[x], g);
        x = g;
        p = ld_parent(&parent[x]);
    }
    return x;
}

__device__ __forceinline__ void uf_unite(uint32_t* parent, uint32_t a, uint32_t b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    while (a != b) {
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicCAS(&parent[a], a, b);   // hook root a under b
        if (old == a) return;
        a = uf_find(parent, old);
        b = uf_find(parent, b);
    }
}

struct Dims {
    uint32_t nx, ny, nz, nxy;
};


// ---- tiled labelling ------------------------------------------------------------
// The grid is cut into 32 x 16 x 16-cell tiles, one workgroup each.  Thread
// j of the workgroup owns local row j (y = j % 16, z = j / 16), 32 cells along
// x as one 32-bit occupancy word.  Inside a tile the components are found with
// a union-find in LDS over the runs of the rows (a row holds at most 16
// runs; run q of row j has index 16 j + q, hooked with LDS CAS); run index
// order is the order of the runs' first keys, so every local root is the
// smallest key of its local component.  Each occupied voxel then stores, as
// its global parent, the rank of its local root.  Adjacencies that cross a
// tile face are hooked afterwards by k_ccl_boundary with the global
// union-find; only those need device-wide atomics.
constexpr int kTX = 32, kTY = 16, kTZ = 16;
constexpr int kTileRows = kTY * kTZ;          // 256 = threads per workgroup
constexpr int kRowRuns = kTX / 2;             // runs per row at most
constexpr int kTileRuns = kTileRows * kRowRuns;   // 4096
static_assert(kTileRows == kBlock, "one thread per tile row");

struct TileGrid {
    uint32_t ntx, nty, ntz;
};

// Workgroups are dealt to the eight XCDs in turn, each with its own L2.  The
// loop index v (v % 8 names its XCD while the grid is a multiple of 8) is
// mapped so that every row of tiles along x (which share bitmap, rank and
// parent lines) is visited on one XCD, and rows go to the XCDs in turn (the
// map's dense regions stay spread over all of them).  Indices past the last
// row map to no tile.
constexpr uint32_t kXcds = 8;

__host__ __device__ inline uint32_t xcd_virtual_tiles(const TileGrid& tg)
{
    const uint32_t rows = tg.nty * tg.ntz;
    return kXcds * tg.ntx * ((rows + kXcds - 1) / kXcds);
}

__device__ __forceinline__ bool xcd_tile(uint32_t v, const TileGrid& tg, uint32_t* t)
{
    const uint32_t x = v % kXcds, i = v / kXcds;
    const uint32_t row = x + kXcds * (i / tg.ntx);
    *t = row * tg.ntx + i % tg.ntx;
    return row < tg.nty * tg.ntz;
}

// 32 occupancy bits of grid row (y, z) starting at x0 (bits beyond NX cleared)
__device__ __forceinline__ uint32_t row_bits(const uint32_t* __restrict__ bits, uint32_t nwords, const Dims& d,
                                             uint32_t x0, uint32_t y, uint32_t z, uint32_t* key0_out)
{
    if (y >= d.ny || z >= d.nz) {
        *key0_out = 0;
        return 0u;
    }
    const uint32_t key0 = x0 + d.nx * (y + d.ny * z);
    *key0_out = key0;
    const uint32_t w = key0 >> 5, sh = key0 & 31;
    uint32_t v = bits[w] >> sh;
    if (sh && w + 1 < nwords) v |= bits[w + 1] << (32 - sh);
    const uint32_t xcount = d.nx - x0 < 32u ? d.nx - x0 : 32u;
    if (xcount < 32u) v &= (1u << xcount) - 1u;
    return v;
}

__device__ __forceinline__ bool bit_at(uint32_t w, int x) { return x >= 0 && x < 32 && ((w >> x) & 1u); }

// first cells of the runs of w, and last cells
__device__ __forceinline__ uint32_t run_starts(uint32_t w) { return w & ~(w << 1); }
__device__ __forceinline__ uint32_t run_ends(uint32_t w) { return w & ~(w >> 1); }

// rank of the first cell of a row segment (occupied cells with smaller keys)
__device__ __forceinline__ uint32_t seg_rank0(const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wrank,
                                              uint32_t key0)
{
    return wrank[key0 >> 5] + __popc(bits[key0 >> 5] & ((1u << (key0 & 31)) - 1u));
}

// Hooks between the runs of row segment v and those of an adjacent row
// segment w (same x range): f(xa, xb) is called for a cell xa of v and an
// adjacent occupied cell xb of w so that every pair of 26-adjacent runs gets
// at least one call.  Two runs touch iff their x ranges, one widened by a
// cell on each side, overlap: an overlap begins where the run of v or the
// run of w starts (first test); a purely diagonal touch is the start of one
// run against the end of the other (second and third tests).  Only run
// starts and ends of v and run starts of w can fire.
template <class F>
__device__ __forceinline__ void hook_segments(uint32_t v, uint32_t w, F&& f)
{
    const uint32_t sv = run_starts(v), ev = run_ends(v);
    for (uint32_t m = v & (sv | ev | run_starts(w)); m; m &= m - 1) {
        const int xl = __ffs(m) - 1;
        const bool st = (sv >> xl) & 1u, en = (ev >> xl) & 1u;
        if (bit_at(w, xl) && (st || !bit_at(w, xl - 1))) f(xl, xl);
        if (st && bit_at(w, xl - 1)) f(xl, xl - 1);
        if (en && bit_at(w, xl + 1)) f(xl, xl + 1);
    }
}

// The calls hook_segments(v, w, f) makes, as masks of the cells xl of v:
// f(xl, xl) for the bits of a, f(xl, xl - 1) for those of b and
// f(xl, xl + 1) for those of c.
struct HookMasks {
    uint32_t a, b, c;
};

__device__ __forceinline__ HookMasks hook_masks(uint32_t v, uint32_t w)
{
    const uint32_t sv = run_starts(v), ev = run_ends(v);
    const uint32_t m = v & (sv | ev | run_starts(w));
    HookMasks h;
    h.a = m & w & (sv | ~(w << 1));
    h.b = m & sv & (w << 1);
    h.c = m & ev & (w >> 1);
    return h;
}

// LDS union-find.  Finds halve the path (a node is re-pointed at its
// grandparent: a store of an ancestor, harmless to concurrent finds), hooks
// put the larger root under the smaller one with a CAS on the root.
__device__ __forceinline__ uint32_t lds_ld(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_find(uint32_t* par, uint32_t x)
{
    uint32_t p = lds_ld(&par[x]);
    while (p != x) {
        const uint32_t g = lds_ld(&par[p]);
        if (g == p) return p;
        lds_st(&par[x], g);
        x = g;
        p = lds_ld(&par[x]);
    }
    return x;
}

// Root of x without writing anything on the way, for when the unions are
// done and other threads are storing roots: a path-halving store could
// replace the root another thread has just stored for a node by an
// intermediate ancestor.
__device__ __forceinline__ uint32_t lds_root(const uint32_t* par, uint32_t x)
{
    uint32_t p = lds_ld(&par[x]);
    while (p != x) {
        x = p;
        p = lds_ld(&par[x]);
    }
    return x;
}

__device__ __forceinline__ void lds_unite(uint32_t* par, uint32_t a, uint32_t b)
{
    a = lds_find(par, a);
    b = lds_find(par, b);
    while (a != b) {
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicCAS(&par[a], a, b);
        if (old == a) return;
        a = lds_find(par, old);
        b = lds_find(par, b);
    }
}

// first cell of the run of w that contains cell x (x must be occupied)
__device__ __forceinline__ uint32_t run_start_of(uint32_t starts, int x)
{
    return 31u - __clz(starts & ((2u << x) - 1u));   // x = 31: (2u << 31) - 1 wraps to all ones
}

// ordinal of that run in its row (runs counted from x = 0)
__device__ __forceinline__ uint32_t run_ordinal(uint32_t starts, int x)
{
    return (uint32_t)__popc(starts & ((2u << x) - 1u)) - 1u;
}

// cell of the n-th (0-based) set bit of w (w has more than n set bits):
// a branch-free binary search over popcounts of halves
__device__ __forceinline__ uint32_t nth_set_bit(uint32_t w, uint32_t n)
{
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t h = 16; h; h >>= 1) {
        const uint32_t c = (uint32_t)__popc(w & ((1u << h) - 1u));
        const bool up = n >= c;
        n -= up ? c : 0u;
        w >>= up ? h : 0u;
        pos += up ? h : 0u;
    }
    return pos;
}

// Hook pairs buffered per tile (more are united in further rounds).  With
// the run table the workgroup holds about 22 KB of LDS, so that seven
// workgroups share a compute unit.
constexpr uint32_t kPairCap = 768;

__global__ void __launch_bounds__(kBlock) k_ccl_tile(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                     const uint32_t* __restrict__ wrank, Dims d, TileGrid tg,
                                                     uint32_t* __restrict__ parent, uint32_t* __restrict__ csize)
{
    __shared__ uint32_t rowv[kTileRows];
    __shared__ uint32_t rowrank[kTileRows];
    __shared__ uint32_t par[kTileRuns];
    __shared__ uint32_t pairs[kPairCap];
    __shared__ uint32_t wtot[kBlock / kWave];
    const uint32_t j = threadIdx.x;
    const int lane = (int)(j & (kWave - 1)), wave = (int)(j / kWave);
    const int yl = (int)(j % kTY), zl = (int)(j / kTY);
    const uint32_t ntiles = tg.ntx * tg.nty * tg.ntz;
    // tiles in the XCD-ordered walk of the face kernel: a row of tiles along
    // x shares its bitmap and rank lines in one L2 (7 % faster than the
    // launch order once the per-run count atomics were gone; with them, the
    // launch order had been faster)
    const uint32_t nv = xcd_virtual_tiles(tg);
    for (uint32_t v0 = blockIdx.x; v0 < nv; v0 += gridDim.x) {
        uint32_t t;
        if (!xcd_tile(v0, tg, &t)) continue;
        const uint32_t tx = t % tg.ntx, ty = (t / tg.ntx) % tg.nty, tz = t / (tg.ntx * tg.nty);
        const uint32_t x0 = tx * kTX, y = ty * kTY + yl, z = tz * kTZ + zl;
        uint32_t key0;
        const uint32_t v = row_bits(bits, nwords, d, x0, y, z, &key0);
        const uint32_t sv = run_starts(v), ev = run_ends(v);
        rowv[j] = v;
        // (unconditional, so that its loads overlap those of the row; rows
        // outside the grid read key 0, and empty rows' ranks are never used)
        rowrank[j] = seg_rank0(bits, wrank, key0);
        // one union-find node per run
        {
            uint32_t c = j * kRowRuns;
            for (uint32_t m = sv; m; m &= m - 1, ++c) par[c] = c;
        }
        // barrier + vote: a tile without occupied cells is skipped by all threads
        if (!__syncthreads_or(v != 0u)) continue;
        // hooks between the runs of the (up to) four neighbouring rows with
        // smaller keys.  Each thread counts its row's hooks from bit masks,
        // a block scan places them in the pair list (plain LDS stores), and
        // all threads then unite the list, so that rows with many hooks do
        // not hold up their wave.  More hooks than the list holds are taken
        // in rounds of kPairCap.
        HookMasks hm[4];
        uint32_t nrow[4];
        uint32_t cnt = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int dy = (q == 0) ? -1 : (q - 2);
            const int dz = (q == 0) ? 0 : -1;
            const int ny2 = yl + dy, nz2 = zl + dz;
            const bool in = v && ny2 >= 0 && ny2 < kTY && nz2 >= 0;
            nrow[q] = in ? (uint32_t)(ny2 + kTY * nz2) : 0u;
            hm[q] = hook_masks(in ? v : 0u, in ? rowv[nrow[q]] : 0u);
            cnt += (uint32_t)(__popc(hm[q].a) + __popc(hm[q].b) + __popc(hm[q].c));
        }
        uint32_t inc = cnt;
#pragma unroll
        for (int dd = 1; dd < kWave; dd <<= 1) {
            const uint32_t o = __shfl_up(inc, dd, kWave);
            if (lane >= dd) inc += o;
        }
        if (lane == kWave - 1) wtot[wave] = inc;
        __syncthreads();
        uint32_t slot = inc - cnt, npairs = 0;
#pragma unroll
        for (int w2 = 0; w2 < kBlock / kWave; ++w2) {
            const uint32_t t2 = wtot[w2];
            slot += (w2 < wave) ? t2 : 0u;
            npairs += t2;
        }
        for (uint32_t r0 = 0; r0 < npairs; r0 += kPairCap) {   // npairs is block-uniform
            if (cnt && slot < r0 + kPairCap && slot + cnt > r0) {
                uint32_t sl = slot;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t nr = nrow[q], sw = run_starts(rowv[nr]);
                    auto put = [&](int xa, int xb) {
                        if (sl >= r0 && sl < r0 + kPairCap) {
                            const uint32_t a = j * kRowRuns + run_ordinal(sv, xa);
                            const uint32_t b = nr * kRowRuns + run_ordinal(sw, xb);
                            pairs[sl - r0] = (a << 16) | b;
                        }
                        ++sl;
                    };
                    for (uint32_t m = hm[q].a; m; m &= m - 1) put(__ffs(m) - 1, __ffs(m) - 1);
                    for (uint32_t m = hm[q].b; m; m &= m - 1) put(__ffs(m) - 1, __ffs(m) - 2);
                    for (uint32_t m = hm[q].c; m; m &= m - 1) put(__ffs(m) - 1, __ffs(m));
                }
            }
            __syncthreads();
            const uint32_t np = min(npairs - r0, kPairCap);
            for (uint32_t i = j; i < np; i += kBlock) {
                const uint32_t pr = pairs[i];
                lds_unite(par, pr >> 16, pr & 0xFFFFu);
            }
            __syncthreads();
        }
        // roots of the runs (a run's entry then holds its root; every value
        // a walk reads is an ancestor or the root) ...
        {
            uint32_t c = j * kRowRuns;
            for (uint32_t m = sv; m; m &= m - 1, ++c) lds_st(&par[c], lds_root(par, c));
        }
        __syncthreads();
        // ... then each run adds its length to its root's count, kept in the
        // upper 16 bits of the root's entry (run indices take 12 bits, a tile
        // holds at most 8192 cells)
        {
            uint32_t c = j * kRowRuns;
            for (uint32_t m = sv; m; m &= m - 1, ++c) {
                const int s0 = __ffs(m) - 1;
                const int e0 = __ffs(ev & ~((1u << s0) - 1u)) - 1;
                atomicAdd(&par[par[c] & 0xFFFFu], (uint32_t)(e0 - s0 + 1) << 16);
            }
        }
        __syncthreads();
        // global parents: the rank of the local root, for a whole run at once
        // (consecutive cells of a run have consecutive ranks); the local
        // root's entry of csize receives its component's voxel count in the
        // tile
        uint32_t c = j * kRowRuns;
        for (uint32_t m = sv; m; m &= m - 1, ++c) {
            const int s0 = __ffs(m) - 1;
            const int e0 = __ffs(ev & ~((1u << s0) - 1u)) - 1;
            const uint32_t pc = par[c], rt = pc & 0xFFFFu;
            const uint32_t rrow = rt / kRowRuns, rx = nth_set_bit(run_starts(rowv[rrow]), rt % kRowRuns);
            const uint32_t rr = rowrank[rrow] + __popc(rowv[rrow] & ((1u << rx) - 1u));
            const uint32_t r = rowrank[j] + __popc(v & ((1u << s0) - 1u));
            // the run's entries: single stores up to a 16-byte boundary, then
            // 16-byte stores, then the rest
            uint32_t p0 = r;
            const uint32_t pe = r + (uint32_t)(e0 - s0 + 1);
            for (; p0 < pe && (p0 & 3u); ++p0) parent[p0] = rr;
            for (; p0 + 4 <= pe; p0 += 4) *reinterpret_cast<uint4*>(parent + p0) = make_uint4(rr, rr, rr, rr);
            for (; p0 < pe; ++p0) parent[p0] = rr;
            // the local root's count, stored once by the tile that owns it (no
            // device atomic: other tiles never write this entry here)
            if (rt == c) csize[r] = pc >> 16;
        }
        // LDS is reused by the next tile (a block with no next tile skips the
        // barrier, which would wait for the stores above to complete)
        if (v0 + gridDim.x < nv) __syncthreads();
    }
}

__device__ __forceinline__ bool occ_cell(const uint32_t* __restrict__ bits, const Dims& d, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= (int)d.nx || y >= (int)d.ny || z >= (int)d.nz) return false;
    return occ(bits, (uint32_t)x + d.nx * ((uint32_t)y + d.ny * (uint32_t)z));
}

// Cross-tile adjacencies, from the cell with the larger key.
//  * y/z faces: a row segment whose neighbouring row (dz = -1 any dy, or
//    dz = 0 and dy = -1) lies in another tile with the same x range hooks the
//    runs of the two segments with the run rule above (runs cut at the tile's
//    x edges are joined inside their tiles).
//  * x faces: the first cell of a segment links each occupied neighbour with
//    a smaller key at x - 1 (five of them), the last cell each one at x + 1
//    (four); these pairs lie in tiles of another x range.
// Each pair is replaced by the local roots of its two voxels (the labelling
// pass left every voxel pointing at its tile-local root), and a tile keeps
// one copy of each distinct root pair (an
// LDS hash set): along a dense surface many cells link the same two local
// components.  The distinct pairs go to the tile's slice of a pair buffer; a
// second kernel unites all pairs of the grid at once.  A tile with more
// distinct pairs than its slice unites the excess itself.
constexpr uint32_t kPairHash = 1024;   // LDS hash set of root pairs per tile
constexpr uint32_t kRawPairs = 1024;   // voxel pairs gathered per tile before the root lookups

__global__ void __launch_bounds__(kBlock) k_ccl_boundary(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                         const uint32_t* __restrict__ wrank, Dims d, TileGrid tg,
                                                         uint32_t* parent, uint64_t* __restrict__ pairs,
                                                         uint32_t* __restrict__ npair)
{
    __shared__ uint64_t raw[kRawPairs];
    __shared__ uint64_t buf[kCclTilePairs];
    __shared__ unsigned long long hset[kPairHash];
    __shared__ uint32_t nbuf;
    const uint32_t j = threadIdx.x;
    const int yl = (int)(j % kTY), zl = (int)(j / kTY);
    // a distinct root pair goes to the tile's list (united in place if full)
    auto add_roots = [&](uint32_t ra, uint32_t rb) {
        const unsigned long long key = ((unsigned long long)ra << 32) | rb;
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 54);   // kPairHash = 2^10 slots
        for (uint32_t probe = 0; probe < kPairHash; ++probe) {
            const unsigned long long old = atomicCAS(&hset[h], ~0ull, key);
            if (old == key) return;          // this root pair is already listed
            if (old == ~0ull) break;         // first time
            h = (h + 1) & (kPairHash - 1);
        }
        const uint32_t i = atomicAdd(&nbuf, 1u);
        if (i < kCclTilePairs) buf[i] = key;
        else uf_unite(parent, ra, rb);
    };
    __shared__ uint32_t wtot[kBlock / kWave];
    const int lane = (int)(j & (kWave - 1)), wave = (int)(j / kWave);
    const uint32_t nv = xcd_virtual_tiles(tg);
    for (uint32_t v0 = blockIdx.x; v0 < nv; v0 += gridDim.x) {
        uint32_t t;
        if (!xcd_tile(v0, tg, &t)) continue;   // uniform over the workgroup
        if (j == 0) nbuf = 0;
        for (uint32_t i = j; i < kPairHash; i += kBlock) hset[i] = ~0ull;
        const uint32_t tx = t % tg.ntx, ty = (t / tg.ntx) % tg.nty, tz = t / (tg.ntx * tg.nty);
        const uint32_t x0 = tx * kTX;
        const int y = (int)(ty * kTY) + yl, z = (int)(tz * kTZ) + zl;
        uint32_t key0;
        const uint32_t v = row_bits(bits, nwords, d, x0, (uint32_t)y, (uint32_t)z, &key0);
        // first the voxel pairs (no loads of parents yet): each thread finds
        // and counts its row's, a block scan places them in the raw list
        const bool face = yl == 0 || yl == kTY - 1 || zl == 0;
        const bool first = (v & 1u) && x0 > 0, last = (v >> 31) & 1u;
        uint32_t r0 = 0, cnt = 0;
        HookMasks hm[4];
        uint32_t fw[4], fn0[4];
        uint32_t fr[5], lr[4], fmask = 0, lmask = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hm[q].a = hm[q].b = hm[q].c = 0;
            fw[q] = fn0[q] = 0;
        }
        if (v && (face || first || last)) {
            r0 = seg_rank0(bits, wrank, key0);
            if (face) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int dy = (q == 0) ? -1 : (q - 2);
                    const int dz = (q == 0) ? 0 : -1;
                    const int ly = yl + dy, lz = zl + dz;
                    if (ly >= 0 && ly < kTY && lz >= 0) continue;   // same tile
                    uint32_t nkey0;
                    const uint32_t w = row_bits(bits, nwords, d, x0, (uint32_t)(y + dy), (uint32_t)(z + dz), &nkey0);
                    if (!w) continue;
                    fw[q] = w;
                    fn0[q] = seg_rank0(bits, wrank, nkey0);
                    hm[q] = hook_masks(v, w);
                    cnt += (uint32_t)(__popc(hm[q].a) + __popc(hm[q].b) + __popc(hm[q].c));
                }
            }
            if (first) {
                const int x = (int)x0;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const int dy = (q < 3) ? q - 1 : (q == 3 ? -1 : 0);
                    const int dz = (q < 3) ? -1 : 0;
                    fr[q] = 0;
                    if (!occ_cell(bits, d, x - 1, y + dy, z + dz)) continue;
                    const uint32_t nk = (uint32_t)(x - 1) + d.nx * ((uint32_t)(y + dy) + d.ny * (uint32_t)(z + dz));
                    fr[q] = rank_of(bits, wrank, nk);
                    fmask |= 1u << q;
                }
            }
            if (last) {
                const int x = (int)x0 + 31;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int dy = (q < 3) ? q - 1 : -1;
                    const int dz = (q < 3) ? -1 : 0;
                    lr[q] = 0;
                    if (!occ_cell(bits, d, x + 1, y + dy, z + dz)) continue;
                    const uint32_t nk = (uint32_t)(x + 1) + d.nx * ((uint32_t)(y + dy) + d.ny * (uint32_t)(z + dz));
                    lr[q] = rank_of(bits, wrank, nk);
                    lmask |= 1u << q;
                }
            }
            cnt += (uint32_t)(__popc(fmask) + __popc(lmask));
        }
        uint32_t inc = cnt;
#pragma unroll
        for (int dd = 1; dd < kWave; dd <<= 1) {
            const uint32_t o = __shfl_up(inc, dd, kWave);
            if (lane >= dd) inc += o;
        }
        if (lane == kWave - 1) wtot[wave] = inc;
        __syncthreads();
        uint32_t slot = inc - cnt, nraw = 0;
#pragma unroll
        for (int w2 = 0; w2 < kBlock / kWave; ++w2) {
            const uint32_t t2 = wtot[w2];
            slot += (w2 < wave) ? t2 : 0u;
            nraw += t2;
        }
        // ... then, a list's worth at a time, the local roots of the pairs,
        // deduplicated (nraw is block-uniform)
        for (uint32_t q0 = 0; q0 < nraw; q0 += kRawPairs) {
            if (cnt && slot < q0 + kRawPairs && slot + cnt > q0) {
                uint32_t sl = slot;
                auto emit = [&](uint32_t a, uint32_t b) {
                    if (sl >= q0 && sl < q0 + kRawPairs) raw[sl - q0] = ((uint64_t)a << 32) | b;
                    ++sl;
                };
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t w = fw[q], n0 = fn0[q];
                    for (uint32_t m = hm[q].a; m; m &= m - 1) {
                        const int xa = __ffs(m) - 1;
                        emit(r0 + __popc(v & ((1u << xa) - 1u)), n0 + __popc(w & ((1u << xa) - 1u)));
                    }
                    for (uint32_t m = hm[q].b; m; m &= m - 1) {
                        const int xa = __ffs(m) - 1;
                        emit(r0 + __popc(v & ((1u << xa) - 1u)), n0 + __popc(w & ((1u << (xa - 1)) - 1u)));
                    }
                    for (uint32_t m = hm[q].c; m; m &= m - 1) {
                        const int xa = __ffs(m) - 1;
                        emit(r0 + __popc(v & ((1u << xa) - 1u)), n0 + __popc(w & ((1u << (xa + 1)) - 1u)));
                    }
                }
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    if ((fmask >> q) & 1u) emit(r0, fr[q]);
                const uint32_t rl = r0 + (uint32_t)__popc(v) - 1u;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if ((lmask >> q) & 1u) emit(rl, lr[q]);
            }
            __syncthreads();
            const uint32_t nr = min(nraw - q0, kRawPairs);
            for (uint32_t i = j; i < nr; i += kBlock) {
                const uint64_t pr = raw[i];
                add_roots(ld_parent(&parent[(uint32_t)(pr >> 32)]), ld_parent(&parent[(uint32_t)pr]));
            }
            __syncthreads();
        }
        const uint32_t np = min(nbuf, kCclTilePairs);
        for (uint32_t i = j; i < np; i += kBlock) pairs[(uint64_t)t * kCclTilePairs + i] = buf[i];
        if (j == 0) npair[t] = np;
        // LDS is reused by the next tile (a block with no next tile skips the
        // barrier, which would wait for the stores above to complete)
        if (v0 + gridDim.x < nv) __syncthreads();
    }
}

// Unions of the buffered cross-tile pairs, one pair per thread.
__global__ void __launch_bounds__(kBlock) k_ccl_pairs(uint32_t ntiles, const uint64_t* __restrict__ pairs,
                                                      const uint32_t* __restrict__ npair, uint32_t* parent)
{
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t np = npair[t];
        for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) {
            const uint64_t pr = pairs[(uint64_t)t * kCclTilePairs + i];
            uf_unite(parent, (uint32_t)(pr >> 32), (uint32_t)pr);
        }
    }
}

// After the merge every tree is final.  Each voxel walks to its root without
// writing anything on the way (a path-halving store here could overwrite the
// root another thread has just stored for that node) and stores only its own
// entry; every value a walk can read is an ancestor, so walks stay correct.
__global__ void __launch_bounds__(kBlock) k_ccl_flatten(const DevCounters* __restrict__ ctr, uint32_t* parent,
                                                        uint32_t* csize)
{
    const uint32_t V = ctr->n_occ;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t stride = gridDim.x * blockDim.x;
    // every lane runs the same iterations (the wave-wide sums below need them all)
    for (uint32_t b0 = blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); b0 < V; b0 += stride) {
        const uint32_t r = b0 + (uint32_t)lane;
        uint32_t x = r, cs = 0;
        if (r < V) {
            // only roots receive counts below, and the count is used only
            // when r is not a root: it can be read before the walk
            const uint32_t own = csize[r];
            const uint32_t p0 = ld_parent(&parent[r]);
            uint32_t p = p0;
            while (p != x) {
                x = p;
                p = ld_parent(&parent[x]);
            }
            if (x != p0) st_parent(&parent[r], x);   // most voxels already point at their root
            // a tile-local root joined to another tile's component hands its
            // count to the component's root (only roots receive counts, so
            // the count read here is final)
            if (x != r) cs = own;
        }
        // one atomic per distinct root in the wave (a large component has
        // many local roots)
        uint64_t pending = __ballot(cs != 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const uint32_t root = __shfl(x, leader, kWave);
            const bool same = cs != 0 && x == root;
            uint32_t v = same ? cs : 0u;
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
            if (lane == leader) atomicAdd(&csize[root], v);
            pending &= ~__ballot(same);
        }
    }
}

// ---- grouping -------------------------------------------------------------------
// One fused scan over the ranks gives, in rank order: the cluster id of each
// kept root (roots of components with at least min_cluster voxels), the
// cluster offsets (running sum of the kept roots' sizes, i.e. clusters in
// label order), and each kept voxel's position among the kept voxels.
struct GroupF {
    const uint32_t* parent;
    const uint32_t* csize;
    uint32_t min_cluster;
    __device__ Vec<3> operator()(uint32_t r) const
    {
        const uint32_t root = parent[r];
        const uint32_t sz = csize[root];
        const bool kept = sz >= min_cluster;
        const bool rt = kept && root == r;
        Vec<3> x;
        x.v[0] = rt ? 1u : 0u;
        x.v[1] = rt ? sz : 0u;
        x.v[2] = kept ? 1u : 0u;
        return x;
    }
};

struct GroupG {
    uint32_t* cid;        // cluster id, at kept roots
    uint32_t* kpos;       // position among kept voxels, at kept voxels
    uint32_t* cl_off;
    uint32_t* cl_tag;
    const uint32_t* occ_key;
    DevCounters* ctr;
    __device__ void operator()(uint32_t r, const Vec<3>& x, const Vec<3>& pre) const
    {
        if (x.v[2]) kpos[r] = pre.v[2];
        if (x.v[0]) {
            cid[r] = pre.v[0];
            cl_off[pre.v[0]] = pre.v[1];
            cl_tag[pre.v[0]] = occ_key[r];
        }
    }
    __device__ void total(const Vec<3>& t) const
    {
        ctr->meta[0] = t.v[0];
        ctr->meta[1] = t.v[1];
        cl_off[t.v[0]] = t.v[1];
        ctr->kmax = t.v[0] ? t.v[0] - 1 : 0;
    }
};

__global__ void __launch_bounds__(kBlock) k_group_pairs(const DevCounters* __restrict__ ctr,
                                                        const uint32_t* __restrict__ parent,
                                                        const uint32_t* __restrict__ csize, uint32_t min_cluster,
                                                        const uint32_t* __restrict__ cid_scan,
                                                        const uint32_t* __restrict__ pos_scan,
                                                        const uint32_t* __restrict__ occ_key,
                                                        uint32_t* __restrict__ out_cid, uint32_t* __restrict__ out_key)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t root = parent[r];
        if (csize[root] >= min_cluster) {
            const uint32_t p = pos_scan[r];
            out_cid[p] = cid_scan[root];
            out_key[p] = occ_key[r];
        }
    }
}

constexpr int kGatherU = 4;

// CSR points: key and Eq. (1) mean of each kept voxel, cluster-major.  Each
// lane gathers kGatherU voxels kGatherU * stride apart, their first probes
// issued together; a probe loads the whole 32-byte slot, so a hit needs no
// second load for the sums.
__global__ void __launch_bounds__(kBlock) k_group_gather(Geom g, Hash h, const DevCounters* __restrict__ ctr,
                                                         const uint32_t* __restrict__ sorted_key0,
                                                         const uint32_t* __restrict__ sorted_key1,
                                                         uint32_t* __restrict__ cl_key, float* __restrict__ cl_x,
                                                         float* __restrict__ cl_y, float* __restrict__ cl_z)
{
    const uint32_t* __restrict__ sorted_key = ctr->group_sel ? sorted_key1 : sorted_key0;
    const uint32_t n = ctr->meta[1];
    const uint32_t nx = (uint32_t)g.dims[0], ny = (uint32_t)g.dims[1];
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t nprobe = h.mask < kMaxProbe ? h.mask + 1u : kMaxProbe;
    for (uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += kGatherU * stride) {
        uint32_t k[kGatherU], s[kGatherU];
        Slot sl[kGatherU];
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const uint32_t i = i0 + (uint32_t)u * stride;
            k[u] = i < n ? sorted_key[i] : kEmpty;
        }
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            s[u] = hash_slot(k[u], h.log2cap);
            if (k[u] != kEmpty) {
                sl[u] = h.slot[s[u]];
            } else {
                sl[u].key = kEmpty;
                sl[u].cnt = 0;
                sl[u].sum[0] = sl[u].sum[1] = sl[u].sum[2] = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const uint32_t i = i0 + (uint32_t)u * stride;
            if (i >= n) continue;
            // linear probing as in hash_find
            for (uint32_t p = 1; sl[u].key != k[u] && sl[u].key != kEmpty && p < nprobe; ++p) {
                s[u] = (s[u] + 1) & h.mask;
                sl[u] = h.slot[s[u]];
            }
            float mx = 0.0f, my = 0.0f, mz = 0.0f;
            if (sl[u].key == k[u]) {
                mx = voxel_mean_axis(k[u] % nx, sl[u].sum[0], sl[u].cnt, g.voxel_size, g.origin[0]);
                my = voxel_mean_axis((k[u] / nx) % ny, sl[u].sum[1], sl[u].cnt, g.voxel_size, g.origin[1]);
                mz = voxel_mean_axis(k[u] / (nx * ny), sl[u].sum[2], sl[u].cnt, g.voxel_size, g.origin[2]);
            }
            cl_key[i] = k[u];
            cl_x[i] = mx;
            cl_y[i] = my;
            cl_z[i] = mz;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_labels(const DevCounters* __restrict__ ctr,
                                                   const uint32_t* __restrict__ parent,
                                                   const uint32_t* __restrict__ occ_key, uint32_t* __restrict__ labels)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x)
        labels[r] = occ_key[parent[r]];
}

Dims dims_of(const Geom& g)
{
    Dims d;
    d.nx = (uint32_t)g.dims[0];
    d.ny = (uint32_t)g.dims[1];
    d.nz = (uint32_t)g.dims[2];
    d.nxy = d.nx * d.ny;
    return d;
}

}  // namespace

uint64_t ccl_tiles(const Geom& g)
{
    const Dims d = dims_of(g);
    return (uint64_t)((d.nx + kTX - 1) / kTX) * ((d.ny + kTY - 1) / kTY) * ((d.nz + kTZ - 1) / kTZ);
}

hipError_t launch_ccl(const Geom& g, const uint32_t* bits, SegBuffers& b, uint32_t cap, DevCounters* ctr,
                      hipStream_t s)
{
    const Dims d = dims_of(g);
    TileGrid tg;
    tg.ntx = (d.nx + kTX - 1) / kTX;
    tg.nty = (d.ny + kTY - 1) / kTY;
    tg.ntz = (d.nz + kTZ - 1) / kTZ;
    const uint64_t ntiles = (uint64_t)tg.ntx * tg.nty * tg.ntz;
    const int tgrid = (int)(ntiles < 16384 ? ntiles : 16384);
    // the labelling and face kernels walk the XCD-ordered tile indices (a
    // multiple of 8, and so is 16384)
    const uint32_t nv = xcd_virtual_tiles(tg);
    const int vgrid = (int)(nv < 16384u ? nv : 16384u);
    {
        StageScope t(VM_STAGE_CCL, s);
        k_ccl_tile<<<vgrid, kBlock, 0, s>>>(bits, g.nwords, b.wrank, d, tg, b.parent, b.csize);
    }
    {
        StageScope t(VM_STAGE_CCL_LINK, s);
        k_ccl_boundary<<<vgrid, kBlock, 0, s>>>(bits, g.nwords, b.wrank, d, tg, b.parent, b.pairs, b.npair);
        k_ccl_pairs<<<tgrid, kBlock, 0, s>>>((uint32_t)ntiles, b.pairs, b.npair, b.parent);
        k_ccl_flatten<<<grid_for(cap), kBlock, 0, s>>>(ctr, b.parent, b.csize);
    }
    return hipGetLastError();
}

hipError_t launch_group(const Geom& g, const Hash& h, SegBuffers& b, uint32_t cap, uint32_t min_cluster,
                        uint32_t* d_labels, DevCounters* ctr, hipStream_t s)
{
    StageScope t(VM_STAGE_GROUP, s);
    const int grid = grid_for(cap);
    if (min_cluster < 1) min_cluster = 1;
    uint32_t* cid = b.scan_a;
    uint32_t* keep = b.sort_k[1];
    const GroupF f{b.parent, b.csize, min_cluster};
    const GroupG gg{cid, keep, b.cl_off, b.cl_tag, b.occ_key, ctr};
    Vec<3>* tiles = reinterpret_cast<Vec<3>*>(b.blk);
    tile_scan<3>(f, gg, &ctr->n_occ, cap, tiles, s);
    hipError_t e;
    k_group_pairs<<<grid, kBlock, 0, s>>>(ctr, b.parent, b.csize, min_cluster, cid, keep, b.occ_key, b.sort_k[0],
                                          b.sort_v[0]);
    // stable sort by cluster id keeps ascending keys inside each cluster
    const uint32_t kbound = cap / min_cluster + 1;
    const int bits_needed = 32 - __builtin_clz(kbound | 1u);
    if ((e = radix_sort_pairs_dev(b.sort_k, b.sort_v, &ctr->meta[1], cap, bits_needed, &ctr->kmax, b.hist, b.blk,
                                  &ctr->group_sel, s)) != hipSuccess)
        return e;
    k_group_gather<<<grid_for((cap + kGatherU - 1) / kGatherU, kBlock, 2048), kBlock, 0, s>>>(
        g, h, ctr, b.sort_v[0], b.sort_v[1], b.cl_key, b.cl_x, b.cl_y, b.cl_z);
    if (d_labels) k_labels<<<grid, kBlock, 0, s>>>(ctr, b.parent, b.occ_key, d_labels);
    return hipGetLastError();
}

}  // namespace vm
