// Stage a1/a2: wrap, leaf binning, Morton keys, stable counting sort by
// (key, original index), per-leaf ranges and the repack into sorted,
// leaf-local coordinates.  Integer work is bit-exact; the FP64 arithmetic
// that decides a leaf index uses explicitly rounded operations (no FMA
// contraction) so that it equals the plain definition
//   w = x - b floor(x / b)  (0 if that gives b),  c = floor(w * (2^L / b)).
#include "fmm_internal.h"
#include "morton.h"
#include "wrap.h"

namespace fmm {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static inline unsigned grid_for(int64_t n, int bs) {
    int64_t g = (n + bs - 1) / bs;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// key[i] and per-leaf counts; flag |= 1 for a non-finite position or charge.
// Wave-aggregated increment of ctr[k]: the active lanes of a wavefront that
// share a key add their number once, and each lane gets the counter's old
// value plus its rank among them (its slot).  Neighbouring atoms usually
// share a leaf, so a wavefront's 64 increments become a few atomics.  Every
// pass serves the key of the first remaining lane, so the loop ends after at
// most 64 passes.
__device__ inline uint32_t wave_agg_inc(uint32_t *ctr, uint32_t k) {
    const int lane = threadIdx.x & 63;
    uint32_t slot = 0;
    bool done = false;
    while (!done) {
        const uint32_t lk = __builtin_amdgcn_readfirstlane(k);
        const unsigned long long m = __ballot(k == lk);
        if (k == lk) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t old = 0;
            if (lane == leader) old = atomicAdd(&ctr[k], (uint32_t)__popcll(m));
            old = __shfl(old, leader);
            slot = old + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            done = true;
        }
    }
    return slot;
}

__global__ void k_bin(int64_t n, const double *__restrict__ pos, const double *__restrict__ q,
                      double box, double scale, uint32_t nc, uint32_t *__restrict__ key,
                      uint32_t *__restrict__ count, int *__restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
        const double qi = q ? q[i] : 0.0;
        if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(qi)) {
            atomicOr(flag, 1);
            key[i] = 0;
            atomicAdd(&count[0], 1u);
            continue;
        }
        const uint32_t cx = leaf_coord(wrap_coord(x, box), scale, nc);
        const uint32_t cy = leaf_coord(wrap_coord(y, box), scale, nc);
        const uint32_t cz = leaf_coord(wrap_coord(z, box), scale, nc);
        const uint32_t k = morton3(cx, cy, cz);
        key[i] = k;
        (void)wave_agg_inc(count, k);
    }
}

hipError_t launch_bin(int64_t n, const double *pos, const double *q, double box, int levels,
                      uint32_t *key, uint32_t *count, int *flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const uint32_t nc = 1u << levels;
    const double scale = (double)nc / box;
    hipLaunchKernelGGL(k_bin, dim3(grid_for(n, 256)), dim3(256), 0, s, n, pos, q, box, scale, nc,
                       key, count, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 counts into int32 starts (out has n + 1 entries).
// Three-phase: per-block scan of 1024 elements, recursive scan of block sums,
// add-back.  Deterministic integer arithmetic.
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;

__global__ void k_scan_block(const uint32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                             int32_t *__restrict__ block_sums) {
    __shared__ int32_t s[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    for (int i = threadIdx.x; i < kScanBlock; i += blockDim.x) {
        int64_t g = base + i;
        s[i] = g < n ? (int32_t)in[g] : 0;
    }
    __syncthreads();
    // Hillis-Steele on 1024 elements with 256 threads (4 per thread)
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int32_t v[4];
        for (int u = 0; u < 4; ++u) {
            int i = threadIdx.x * 4 + u;
            v[u] = i >= off ? s[i - off] : 0;
        }
        __syncthreads();
        for (int u = 0; u < 4; ++u) s[threadIdx.x * 4 + u] += v[u];
        __syncthreads();
    }
    for (int i = threadIdx.x; i < kScanBlock; i += blockDim.x) {
        int64_t g = base + i;
        if (g < n) out[g] = (i == 0 ? 0 : s[i - 1]);  // exclusive
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s[kScanBlock - 1];
}

__global__ void k_scan_add(int32_t *__restrict__ out, int64_t n, const int32_t *__restrict__ offs) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    const int32_t o = offs[blockIdx.x];
    for (int i = threadIdx.x; i < kScanBlock; i += blockDim.x) {
        int64_t g = base + i;
        if (g < n) out[g] += o;
    }
}

__global__ void k_set_total(int32_t *out, int64_t n, const uint32_t *in) {
    // out[n] = out[n-1] + in[n-1]
    if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = (n > 0 ? out[n - 1] + (int32_t)in[n - 1] : 0);
}

int64_t scan_scratch_len(int64_t n) {
    int64_t total = 0;
    int64_t m = n;
    while (m > 1) {
        int64_t nb = (m + kScanBlock - 1) / kScanBlock;
        total += 2 * nb + 2;
        m = nb;
    }
    return total + 4;
}

// scratch: int32 buffer of scan_scratch_len(n)
static hipError_t scan_rec(const uint32_t *in_u, const int32_t *in_i, int32_t *out, int64_t n,
                           int32_t *scratch, hipStream_t s);

__global__ void k_scan_block_i(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                               int32_t *__restrict__ block_sums) {
    __shared__ int32_t s[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    for (int i = threadIdx.x; i < kScanBlock; i += blockDim.x) {
        int64_t g = base + i;
        s[i] = g < n ? in[g] : 0;
    }
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int32_t v[4];
        for (int u = 0; u < 4; ++u) {
            int i = threadIdx.x * 4 + u;
            v[u] = i >= off ? s[i - off] : 0;
        }
        __syncthreads();
        for (int u = 0; u < 4; ++u) s[threadIdx.x * 4 + u] += v[u];
        __syncthreads();
    }
    for (int i = threadIdx.x; i < kScanBlock; i += blockDim.x) {
        int64_t g = base + i;
        if (g < n) out[g] = (i == 0 ? 0 : s[i - 1]);
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = s[kScanBlock - 1];
}

static hipError_t scan_rec(const uint32_t *in_u, const int32_t *in_i, int32_t *out, int64_t n,
                           int32_t *scratch, hipStream_t s) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    int32_t *sums = scratch;
    int32_t *sums_scan = scratch + nb + 1;
    int32_t *rest = scratch + 2 * nb + 2;
    if (in_u)
        hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(256), 0, s, in_u, out, n, sums);
    else
        hipLaunchKernelGGL(k_scan_block_i, dim3((unsigned)nb), dim3(256), 0, s, in_i, out, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    e = scan_rec(nullptr, sums, sums_scan, nb, rest, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, out, n, sums_scan);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                       int64_t scratch_len, hipStream_t s) {
    if (scratch_len < scan_scratch_len(n)) return hipErrorInvalidValue;
    if (n > 0) {
        hipError_t e = scan_rec(in, nullptr, out, n, scratch, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_set_total, dim3(1), dim3(64), 0, s, out, n, in);
    return hipGetLastError();
}

// Scatter original indices into their leaf segment (order inside a segment
// is then fixed by k_cell_sort).
__global__ void k_scatter(int64_t n, const uint32_t *__restrict__ key, const int32_t *__restrict__ start,
                          uint32_t *__restrict__ cursor, int32_t *__restrict__ perm) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = key[i];
        const uint32_t slot = wave_agg_inc(cursor, k);
        perm[start[k] + (int32_t)slot] = (int32_t)i;
    }
}

hipError_t launch_scatter(int64_t n, const uint32_t *key, const int32_t *start, uint32_t *cursor,
                          int32_t *perm, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, n, key, start, cursor, perm);
    return hipGetLastError();
}

// Order each leaf segment by original index: makes the order (key, index),
// i.e. a stable sort, independent of atomic arrival order.  One wavefront
// per leaf: the segment is staged in LDS and every lane places its entries
// by rank (the number of smaller indices in the segment; indices are
// distinct), so the cost is n^2/64 compares per leaf instead of a serial
// insertion sort.  Segments longer than kSortCap (degenerate inputs) are
// sorted by lane 0 by insertion.
constexpr int kSortCap = 1024;

__global__ __launch_bounds__(256) void k_cell_sort(int64_t nleaf, const int32_t *__restrict__ start,
                                                   int32_t *__restrict__ perm) {
    __shared__ int32_t buf[4][kSortCap];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + w));
    if (c >= nleaf) return;  // whole wavefront; no block barriers below
    const int32_t b = start[c], n = start[c + 1] - b;
    if (n <= 1) return;
    if (n > kSortCap) {
        if (lane == 0)
            for (int32_t i = b + 1; i < b + n; ++i) {
                const int32_t v = perm[i];
                int32_t j = i - 1;
                while (j >= b && perm[j] > v) {
                    perm[j + 1] = perm[j];
                    --j;
                }
                perm[j + 1] = v;
            }
        return;
    }
    int32_t *sb = buf[w];
    for (int32_t i = lane; i < n; i += 64) sb[i] = perm[b + i];
    // LDS accesses of one wavefront complete in order; the fence keeps the
    // compiler from moving the reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int32_t i = lane; i < n; i += 64) {
        const int32_t v = sb[i];
        int32_t r = 0;
        for (int32_t j = 0; j < n; ++j) r += sb[j] < v ? 1 : 0;
        perm[b + r] = v;
    }
}

hipError_t launch_cell_sort(int64_t nleaf, const int32_t *start, int32_t *perm, hipStream_t s) {
    if (nleaf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)((nleaf + 3) / 4)), dim3(256), 0, s, nleaf, start, perm);
    return hipGetLastError();
}

// Repack in sorted order: leaf-local coordinates (x - leaf centre) and
// charge in the mode's precision (xq), plus an FP64 copy (xs) of the wrapped
// position measured from the box centre and the charge, which the correction
// terms, the energy reduction and the solute-solvent pass read later (so
// they never touch the caller's arrays again).
template <typename T>
__global__ void k_gather(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ pos,
                         const double *__restrict__ q, double box, double scale, uint32_t nc, double h,
                         T *__restrict__ xq, double *__restrict__ xs) {
    const double hb = 0.5 * box;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = perm[s];
        double w[3];
        double loc[3];
        for (int a = 0; a < 3; ++a) {
            w[a] = wrap_coord(pos[3 * (int64_t)i + a], box);
            const uint32_t c = leaf_coord(w[a], scale, nc);
            loc[a] = w[a] - ((double)c + 0.5) * h;
        }
        const double qi = q[i];
        xq[4 * s + 0] = (T)loc[0];
        xq[4 * s + 1] = (T)loc[1];
        xq[4 * s + 2] = (T)loc[2];
        xq[4 * s + 3] = (T)qi;
        xs[4 * s + 0] = w[0] - hb;
        xs[4 * s + 1] = w[1] - hb;
        xs[4 * s + 2] = w[2] - hb;
        xs[4 * s + 3] = qi;
    }
}

hipError_t launch_gather(int64_t n, const int32_t *perm, const double *pos, const double *q, double box,
                         int levels, bool fp64, void *xq, double *xs, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const uint32_t nc = 1u << levels;
    const double scale = (double)nc / box;
    const double h = box / (double)nc;
    if (fp64)
        hipLaunchKernelGGL(k_gather<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, pos, q, box,
                           scale, nc, h, (double *)xq, xs);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, pos, q, box,
                           scale, nc, h, (float *)xq, xs);
    return hipGetLastError();
}

// Near-field copy of xq with every leaf padded to a multiple of G atoms
// (G = source groups of the P2P kernel), so the P2P inner loop needs no
// per-lane bounds test.  Padding atoms have q = 0 and sit far outside the
// leaf, where their terms vanish
// without forming 0/0 (leaf-local coordinate `far` per axis, chosen by the
// caller well beyond the reach of any shifted neighbour).
// pcount[c] = round_up(count[c], G).
__global__ void k_pad_counts(int64_t nleaf, const uint32_t *__restrict__ count, uint32_t G,
                             uint32_t *__restrict__ pcount) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nleaf;
         c += (int64_t)gridDim.x * blockDim.x)
        pcount[c] = (count[c] + G - 1) / G * G;
}

hipError_t launch_pad_counts(int64_t nleaf, const uint32_t *count, int G, uint32_t *pcount, hipStream_t s) {
    if (nleaf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_counts, dim3(grid_for(nleaf, 256)), dim3(256), 0, s, nleaf, count, (uint32_t)G,
                       pcount);
    return hipGetLastError();
}

// one wavefront per leaf; lanes copy the leaf's slots
template <typename T>
__global__ __launch_bounds__(256) void k_pad_gather(int64_t nleaf, const int32_t *__restrict__ start,
                                                    const int32_t *__restrict__ pstart, const T *__restrict__ xq,
                                                    T far, T *__restrict__ xqp) {
    const int64_t leaf = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (leaf >= nleaf) return;
    const int lane = threadIdx.x & 63;
    const int32_t s0 = start[leaf], cnt = start[leaf + 1] - s0;
    const int32_t p0 = pstart[leaf], pcnt = pstart[leaf + 1] - p0;
    for (int32_t t = lane; t < pcnt; t += 64) {
        T *d = xqp + 4 * (int64_t)(p0 + t);
        if (t < cnt) {
            const T *src = xq + 4 * (int64_t)(s0 + t);
            d[0] = src[0];
            d[1] = src[1];
            d[2] = src[2];
            d[3] = src[3];
        } else {
            d[0] = far;
            d[1] = far;
            d[2] = far;
            d[3] = (T)0;
        }
    }
}

hipError_t launch_pad_gather(int64_t nleaf, const int32_t *start, const int32_t *pstart, bool fp64,
                             const void *xq, double far, void *xqp, hipStream_t s) {
    if (nleaf <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((nleaf + 3) / 4);
    if (fp64)
        hipLaunchKernelGGL(k_pad_gather<double>, dim3(grid), dim3(256), 0, s, nleaf, start, pstart,
                           (const double *)xq, far, (double *)xqp);
    else
        hipLaunchKernelGGL(k_pad_gather<float>, dim3(grid), dim3(256), 0, s, nleaf, start, pstart,
                           (const float *)xq, (float)far, (float *)xqp);
    return hipGetLastError();
}

// Solute-only charges for the second far-field pass of the solute-solvent
// scheme: xq_u = xq with q multiplied by the solute flag of the atom.
template <typename T>
__global__ void k_mask_charges(int64_t n, const int32_t *__restrict__ perm, const uint8_t *__restrict__ mask,
                               const T *__restrict__ xq, T *__restrict__ xq_u) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const bool u = mask[perm[s]] != 0;
        xq_u[4 * s + 0] = xq[4 * s + 0];
        xq_u[4 * s + 1] = xq[4 * s + 1];
        xq_u[4 * s + 2] = xq[4 * s + 2];
        xq_u[4 * s + 3] = u ? xq[4 * s + 3] : (T)0;
    }
}

hipError_t launch_mask_charges(int64_t n, const int32_t *perm, const uint8_t *mask, bool fp64, const void *xq,
                               void *xq_u, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_mask_charges<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, mask,
                           (const double *)xq, (double *)xq_u);
    else
        hipLaunchKernelGGL(k_mask_charges<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, mask,
                           (const float *)xq, (float *)xq_u);
    return hipGetLastError();
}

// out[i] = 1 - (mask[i] != 0): the solvent as the masked set
__global__ void k_invert_mask(int64_t n, const uint8_t *__restrict__ mask, uint8_t *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = mask[i] ? 0 : 1;
}

hipError_t launch_invert_mask(int64_t n, const uint8_t *mask, uint8_t *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_invert_mask, dim3(grid_for(n, 256)), dim3(256), 0, s, n, mask, out);
    return hipGetLastError();
}

}  // namespace fmm
