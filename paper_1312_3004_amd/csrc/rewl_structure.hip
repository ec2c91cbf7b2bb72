// rewl_structure.hip -- structural observables of lipid configurations
// (Sec. 3.2, Eqs. 6-8): the bond order parameter S_mol of the head bonds, the
// clusters of lipids whose tails touch, and the gyration tensor and
// prolateness of the largest cluster in unfolded coordinates.
//
// One workgroup of four wavefronts per configuration.  The lipid beads go to
// LDS; the contact graph is held as one bit row per lipid, built 64 partners
// at a time with a ballot, each pair tested once (the rows are shared among
// the four wavefronts, the blocks left of the diagonal filled by transposing
// bits).  Then wavefront 0 alone takes S_mol, grows the clusters level by
// level (visited set, frontier and each level's finds as register bit
// masks), unfolds the largest one level by level in binary64 and reduces it.
// Sums across lanes use butterfly shuffles, so the floating-point outputs
// agree with a plain evaluation to rounding, while every integer output
// (cluster count and sizes, the tree that unfolds a cluster) is decided as in
// the definition (binary32 minimum images, binary64 squared distances, a
// binary32 screen settling only the pairs it provably can) and is exact.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rewl_host.h"

namespace rewl_gpu {

namespace {

constexpr int kStructMaxLipids = 512;
constexpr int kStructWords = kStructMaxLipids / 64;
constexpr double kTailContact2 = 1.96;   // (1.4 sigma)^2
constexpr int kStructWaves = 4;          // wavefronts per configuration for the contact rows

// Orders a wavefront's own LDS writes before its later reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// b - a moved once by -+box when beyond +-box/2 (selects, no branches).
__device__ __forceinline__ double st_min_image(float a, float b, float box, float half) {
    const float x = b - a;
    const float lo = x - box, hi = x + box;
    return (double)(x > half ? lo : (x < -half ? hi : x));
}

__device__ __forceinline__ void st_diff(const float *a, const float *b, float box, float half, double d[3]) {
    d[0] = st_min_image(a[0], b[0], box, half);
    d[1] = st_min_image(a[1], b[1], box, half);
    d[2] = st_min_image(a[2], b[2], box, half);
}

__device__ __forceinline__ double st_r2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ bool tails_touch(const float *xi, const float *xj, float box, float half) {
    // xi, xj: the lipid's three beads (head, centre, end) as 9 floats.
    double d[3];
    int hit = 0;
#pragma unroll
    for (int a = 1; a < 3; ++a)
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            st_diff(xi + 3 * a, xj + 3 * b, box, half, d);
            hit |= (int)(st_r2(d) < kTailContact2);
        }
    return hit != 0;
}

// The same decision from binary32 squared distances where they settle it:
// fl32((dx^2 + dy^2) + dz^2) of the binary32 differences is within 3 ulp
// (1.8e-7 relative) of the exact sum, and the binary64 sum within 2.3e-16, so
// a value below 1.959997 (1.96 (1 - 1.5e-6)) is a contact and one above
// 1.960003 is not.  *unsure is set when a pair falls between (NaN never
// does); the caller then takes tails_touch.
__device__ __forceinline__ bool tails_touch_fast(const float *xi, const float *xj, float box, float half,
                                                 bool *unsure) {
    int hit = 0, amb = 0;
#pragma unroll
    for (int a = 1; a < 3; ++a)
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            float d[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float x = xj[3 * b + c] - xi[3 * a + c];
                const float lo = x - box, hi = x + box;
                d[c] = x > half ? lo : (x < -half ? hi : x);
            }
            const float r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            hit |= (int)(r2 < 1.959997f);
            amb |= (int)(r2 >= 1.959997f && r2 <= 1.960003f);
        }
    *unsure = amb != 0;
    return hit != 0;
}

// Place the beads of a lipid other than `b` through its bonds, starting from
// bead b (0 head, 1 centre, 2 end) already at u[3 b].
__device__ __forceinline__ void st_chain(const float *x, double *u, int b, float box, float half) {
    double d[3];
    if (b == 1) {
        st_diff(x + 3, x, box, half, d);
        for (int a = 0; a < 3; ++a) u[a] = u[3 + a] + d[a];
        st_diff(x + 3, x + 6, box, half, d);
        for (int a = 0; a < 3; ++a) u[6 + a] = u[3 + a] + d[a];
    } else if (b == 2) {
        st_diff(x + 6, x + 3, box, half, d);
        for (int a = 0; a < 3; ++a) u[3 + a] = u[6 + a] + d[a];
        st_diff(x + 3, x, box, half, d);
        for (int a = 0; a < 3; ++a) u[a] = u[3 + a] + d[a];
    } else {
        st_diff(x, x + 3, box, half, d);
        for (int a = 0; a < 3; ++a) u[3 + a] = u[a] + d[a];
        st_diff(x + 3, x + 6, box, half, d);
        for (int a = 0; a < 3; ++a) u[6 + a] = u[3 + a] + d[a];
    }
}

// LDS layout for M lipids (W = ceil(M / 64) mask words):
//   xs  float [M][9]      bead coordinates (head, centre, end)
//   adj u64   [M][W]      contact rows
//   u   double[M][9]      unfolded beads of the largest cluster
//   root, level, parent int32[M]
__global__ __launch_bounds__(256) void k_lipid_structure(const unsigned char *xbase, size_t xstride,
                                                       const unsigned char *lbase, size_t lstride, int np, int M,
                                                       float box, double *out) {
    extern __shared__ __align__(16) unsigned char st_lds[];
    const int W = (M + 63) >> 6;
    uint64_t *adj = (uint64_t *)st_lds;
    double *u = (double *)(adj + (size_t)M * W);
    float *xs = (float *)(u + (size_t)M * 9);
    int *root = (int *)(xs + (size_t)M * 9);
    int *level = root + M;
    int *parent = level + M;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int c = blockIdx.x;
    const float half = 0.5f * box;
    const float *x = (const float *)(xbase + (size_t)c * xstride);
    const int32_t *lp = (const int32_t *)(lbase + (size_t)c * lstride);
    double *rec = out + (size_t)c * 8;

    // Beads to LDS; an index outside [0, np) turns the record into NaN.
    bool bad = false;
    for (int l = tid; l < M; l += 64 * kStructWaves) {
        for (int b = 0; b < 3; ++b) {
            const int p = lp[3 * l + b];
            const bool ok = p >= 0 && p < np;
            bad = bad || !ok;
            const int q = ok ? p : 0;
            for (int a = 0; a < 3; ++a) xs[9 * l + 3 * b + a] = x[3 * (size_t)q + a];
        }
        root[l] = -1;
    }
    if (__syncthreads_or(bad)) {
        if (tid < 8) rec[tid] = __builtin_nan("");
        return;
    }

    // Contact rows: row i, word w holds partners j = 64 w + lane; wavefront v
    // builds rows i = v mod 4, words from the one holding i onwards (the test
    // is symmetric in i and j).  Each lane keeps its own lipid's beads in
    // registers (NaN past the end, which never touches) and reads lipid i's,
    // the same address for all lanes.
    for (int w = 0; w < W; ++w) {
        const int j = 64 * w + lane;
        float tj[9];
        for (int a = 0; a < 9; ++a) tj[a] = j < M ? xs[9 * j + a] : __builtin_nanf("");
        for (int i = wave; i < M && (i >> 6) <= w; i += kStructWaves) {
            bool unsure;
            bool hit = tails_touch_fast(xs + 9 * i, tj, box, half, &unsure);
            if (__any(unsure)) hit = tails_touch(xs + 9 * i, tj, box, half);
            const uint64_t m = __ballot(hit & (j != i));
            if (lane == 0) adj[(size_t)i * W + w] = m;
        }
    }
    __syncthreads();
    // Words left of row i's own block, by transposing: bit j of row i is bit
    // i of row j, a word already built above.
    for (int i = 64 + wave; i < M; i += kStructWaves) {
        for (int w = 0; w < (i >> 6); ++w) {
            const int j = 64 * w + lane;
            const bool hit = (adj[(size_t)j * W + (i >> 6)] >> (i & 63)) & 1ull;
            const uint64_t m = __ballot(hit);
            if (lane == 0) adj[(size_t)i * W + w] = m;
        }
    }
    __syncthreads();
    // The rest runs on wavefront 0 alone: the others leave after the last
    // workgroup barrier, and wavefront 0 orders its LDS traffic with
    // wave-level fences from here on.
    if (wave != 0) return;

    // Eq. 6: <cos^2> of the head-to-centre bonds along each axis.
    double cx = 0.0, cy = 0.0, cz = 0.0;
    for (int l = lane; l < M; l += 64) {
        double d[3];
        st_diff(xs + 9 * l, xs + 9 * l + 3, box, half, d);
        const double r2 = st_r2(d);
        cx += d[0] * d[0] / r2;
        cy += d[1] * d[1] / r2;
        cz += d[2] * d[2] / r2;
    }
    cx = wave_sum(cx);
    cy = wave_sum(cy);
    cz = wave_sum(cz);

    // Clusters, grown breadth first from their lowest free lipid.  The
    // visited set and the frontier are bit masks held by every lane alike;
    // the search reads only the contact rows and writes root, level and
    // parent for the unfolding, so it needs no LDS ordering.
    uint64_t vis[kStructWords], front[kStructWords];
#pragma unroll
    for (int w = 0; w < kStructWords; ++w) {
        const int left = M - 64 * w;   // lipids in word w
        vis[w] = left >= 64 ? 0ull : (left <= 0 ? ~0ull : ~((1ull << left) - 1ull));
        front[w] = 0ull;
    }
    int ncl = 0, best_root = -1, best_size = 0, best_depth = 0;
    for (;;) {
        int r = -1;
#pragma unroll
        for (int w = kStructWords - 1; w >= 0; --w)
            if (~vis[w]) r = 64 * w + __builtin_ctzll(~vis[w]);
        if (r < 0) break;
        ++ncl;
        if (lane == 0) {
            root[r] = r;
            level[r] = 0;
            parent[r] = -1;
        }
#pragma unroll
        for (int w = 0; w < kStructWords; ++w) {
            front[w] = w == (r >> 6) ? 1ull << (r & 63) : 0ull;
            vis[w] |= front[w];
        }
        int size = 1, k = 0;
        for (;;) {
            uint64_t found[kStructWords];
            int nfound = 0;
#pragma unroll
            for (int w = 0; w < kStructWords; ++w) {
                found[w] = 0ull;
                if (w < W) {
                    const int j = 64 * w + lane;
                    int p = -1;
                    if (!((vis[w] >> lane) & 1ull)) {   // free, and j < M
#pragma unroll
                        for (int v = 0; v < kStructWords; ++v) {
                            if (v < W) {
                                const uint64_t t = adj[(size_t)j * W + v] & front[v];
                                if (p < 0 && t) p = 64 * v + __builtin_ctzll(t);
                            }
                        }
                    }
                    found[w] = __ballot(p >= 0);
                    if (p >= 0) {
                        root[j] = r;
                        level[j] = k + 1;
                        parent[j] = p;
                    }
                    nfound += __builtin_popcountll(found[w]);
                }
            }
            if (nfound == 0) break;
            size += nfound;
            ++k;
#pragma unroll
            for (int w = 0; w < kStructWords; ++w) {
                front[w] = found[w];
                vis[w] |= found[w];
            }
        }
        if (size > best_size) {
            best_size = size;
            best_root = r;
            best_depth = k;
        }
    }
    wave_sync();

    // Unfold the largest cluster level by level.
    for (int k = 0; k <= best_depth; ++k) {
        for (int j = lane; j < M; j += 64) {
            if (root[j] != best_root || level[j] != k) continue;
            const float *xj = xs + 9 * j;
            double *uj = u + 9 * j;
            if (k == 0) {
                for (int a = 0; a < 3; ++a) uj[a] = (double)xj[a];
                st_chain(xj, uj, 0, box, half);
                continue;
            }
            const int i = parent[j];
            const float *xi = xs + 9 * i;
            const double *ui = u + 9 * i;
            int b = 0;
            for (int pr = 0; pr < 4 && b == 0; ++pr) {
                const int ba = 1 + (pr >> 1), bb = 1 + (pr & 1);
                double d[3];
                st_diff(xi + 3 * ba, xj + 3 * bb, box, half, d);
                if (st_r2(d) < kTailContact2) {
                    for (int a = 0; a < 3; ++a) uj[3 * bb + a] = ui[3 * ba + a] + d[a];
                    b = bb;
                }
            }
            st_chain(xj, uj, b, box, half);
        }
        wave_sync();
    }

    // Eq. 7 over the 3 x best_size beads, then Eq. 8.
    double s[3] = {0.0, 0.0, 0.0};
    for (int j = lane; j < M; j += 64) {
        if (root[j] != best_root) continue;
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) s[a] += u[9 * j + 3 * b + a];
    }
    const double n = 3.0 * (double)best_size;
    double com[3], q[3];
    for (int a = 0; a < 3; ++a) com[a] = wave_sum(s[a]) / n;
    for (int a = 0; a < 3; ++a) s[a] = 0.0;
    for (int j = lane; j < M; j += 64) {
        if (root[j] != best_root) continue;
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double e = u[9 * j + 3 * b + a] - com[a];
                s[a] += e * e;
            }
    }
    for (int a = 0; a < 3; ++a) q[a] = wave_sum(s[a]) / n;

    if (lane == 0) {
        const double sx = 1.5 * (cx / (double)M) - 0.5;
        const double sy = 1.5 * (cy / (double)M) - 0.5;
        const double sz = 1.5 * (cz / (double)M) - 0.5;
        double smax = sx;
        int axis = 0;
        if (sy > smax) { smax = sy; axis = 1; }
        if (sz > smax) { smax = sz; axis = 2; }
        const double tr = q[0] + q[1] + q[2];
        const double lam = tr / 3.0;
        const double e0 = q[0] - lam, e1 = q[1] - lam, e2 = q[2] - lam;
        const double num = e0 * e0 * e0 + e1 * e1 * e1 + e2 * e2 * e2;
        rec[0] = smax;
        rec[1] = (double)axis;
        rec[2] = (double)ncl;
        rec[3] = (double)best_size;
        rec[4] = q[0];
        rec[5] = q[1];
        rec[6] = q[2];
        rec[7] = 9.0 * num / (tr * tr * tr);
    }
}

// H(E, O) of the lipid model at a sync point (Sec. 3.2), one thread per
// walker, from the record just computed: O = lipids in the largest cluster
// (field 3), O bin O obs_bins / (nlip + 1); or, for a floating-point field v,
// O = its bin floor((v - lo) / (hi - lo) * obs_bins) held to [0, obs_bins).
// The sample goes to the walker's energy bin within its window (each walker
// owns its cells: no atomics).
__global__ __launch_bounds__(64) void k_measure_lipid(DevState st) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= st.nw || *st.converged) return;
    const int b = st.E[w] - st.start[w / st.m];
    if (b < 0 || b >= st.W) return;
    int O, ob;
    if (st.obs_field == 3) {
        const double v = st.obs_rec[(size_t)w * 8 + 3];
        if (!(v >= 1.0 && v <= (double)st.nmol)) return;   // only a NaN record (never in a run)
        O = (int)v;
        ob = (int)(((long long)O * st.obs_bins) / (st.nmol + 1));
    } else {
        const double v = st.obs_rec[(size_t)w * 8 + st.obs_field];
        const double t = (v - st.obs_lo) / (st.obs_hi - st.obs_lo) * (double)st.obs_bins;
        O = t >= 0.0 ? (t < (double)st.obs_bins ? (int)t : st.obs_bins - 1) : 0;
        ob = O;
    }
    const size_t cell = (size_t)w * st.Wpad + b;
    st.obs_hist[cell * st.obs_bins + ob] += 1u;
    st.obs_sum[cell] += (unsigned long long)O;
    st.obs_cnt[cell] += 1u;
}

}  // namespace

size_t lipid_structure_lds_bytes(int M) {
    const size_t W = (size_t)(M + 63) / 64;
    return (size_t)M * W * 8 + (size_t)M * 72 + (size_t)M * 36 + (size_t)M * 12;
}

hipError_t launch_lipid_structure(const void *coords, size_t xstride, const void *lipids, size_t lstride, int nconf,
                                  int np, int M, float box, double *out, hipStream_t s) {
    const size_t lds = lipid_structure_lds_bytes(M);
    if (lds > 48 * 1024) {   // with margin for the kernel's own static LDS
        const hipError_t e = hipFuncSetAttribute((const void *)k_lipid_structure,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_lipid_structure, dim3(nconf), dim3(64 * kStructWaves), lds, s,
                       (const unsigned char *)coords, xstride, (const unsigned char *)lipids, lstride, np, M, box, out);
    return hipGetLastError();
}

hipError_t launch_lipid_measure(const DevState &st, hipStream_t s) {
    const unsigned char *rows = (const unsigned char *)st.spins;
    hipError_t e = launch_lipid_structure(rows, (size_t)st.Npad, rows + st.lip_off_lip, (size_t)st.Npad, st.nw, st.nb,
                                          st.nmol, st.box, st.obs_rec, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_measure_lipid, dim3((unsigned)((st.nw + 63) / 64)), dim3(64), 0, s, st);
    return hipGetLastError();
}

}  // namespace rewl_gpu

using rewl_host::fail;

static int check_structure_args(int nconf, int np, int nlip, float box) {
    if (nconf < 0) return fail(REWL_EINVAL, "nconf must be >= 0");
    if (nlip < 1 || nlip > rewl_gpu::kStructMaxLipids) return fail(REWL_EINVAL, "nlip must be in [1, 512]");
    if (np < 3 * nlip) return fail(REWL_EINVAL, "np must be >= 3 nlip");
    if (!(box > 0.0f) || !(box < 1e30f)) return fail(REWL_EINVAL, "box must be positive and finite");
    return REWL_OK;
}

extern "C" int rewl_lipid_structure(const float *coords, size_t coord_stride, const int32_t *lipids,
                                    size_t lipid_stride, int nconf, int np, int nlip, float box, double *out,
                                    void *hip_stream) {
    int st = check_structure_args(nconf, np, nlip, box);
    if (st != REWL_OK) return st;
    if (nconf == 0) return REWL_OK;
    if (!coords || !lipids || !out) return fail(REWL_EINVAL, "null pointer");
    if (((uintptr_t)coords & 3) || ((uintptr_t)lipids & 3) || ((uintptr_t)out & 7) || (coord_stride & 3) ||
        (lipid_stride & 3))
        return fail(REWL_EINVAL, "coords and lipids must be 4-byte aligned (strides too), out 8-byte aligned");
    if (nconf > 1 && (coord_stride < (size_t)12 * np || lipid_stride < (size_t)12 * nlip))
        return fail(REWL_EINVAL, "strides smaller than one configuration");
    HIP_TRY(rewl_gpu::launch_lipid_structure(coords, coord_stride, lipids, lipid_stride, nconf, np, nlip, box, out,
                                             (hipStream_t)hip_stream));
    return REWL_OK;
}

extern "C" int rewl_lipid_obs_field(rewl_t *r, int field, double lo, double hi) {
    if (!r) return fail(REWL_EINVAL, "null handle");
    rewl_gpu::DevState &d = r->st;
    if (d.model != rewl_gpu::kModelLipid3D) return fail(REWL_EINVAL, "not a run of the lipid model");
    if (d.obs_bins <= 0) return fail(REWL_EINVAL, "the run samples no observable (opts.obs_bins = 0)");
    if (field == 3) {
        d.obs_field = 3;
        d.obs_lo = d.obs_hi = 0.0;
        return REWL_OK;
    }
    if (field != 0 && (field < 4 || field > 7)) return fail(REWL_EINVAL, "field must be 0, 3, 4, 5, 6 or 7");
    if (!(lo > -1e300 && hi < 1e300 && hi > lo)) return fail(REWL_EINVAL, "need finite lo < hi");
    d.obs_field = field;
    d.obs_lo = lo;
    d.obs_hi = hi;
    return REWL_OK;
}

// Record buffer of rewl_structure_noalloc: a file-scope device array (one
// copy on every GPU the library runs on, held until the process ends) for
// callers that cannot allocate device memory.  Host code never passes the
// array's name to a kernel: it takes the device address of each GPU's copy
// once, with that GPU current, and passes that address.
constexpr int kNoallocMaxWalkers = 4096;
static __device__ __align__(256) double scratch[kNoallocMaxWalkers * 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of GPU `dev`'s copy of `scratch`.
int scratch_on(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(REWL_EDEVICE, "device index beyond the record buffers kept");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(REWL_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return REWL_OK;
}
}  // namespace

extern "C" int rewl_structure_noalloc(rewl_t *r, double *out) {
    if (!r || !out) return fail(REWL_EINVAL, "null argument");
    const rewl_gpu::DevState &d = r->st;
    if (d.model != rewl_gpu::kModelLipid3D) return fail(REWL_EINVAL, "not a run of the lipid model");
    int st = check_structure_args(d.nw, d.nb, d.nmol, d.box);
    if (st != REWL_OK) return st;
    if (d.nw > kNoallocMaxWalkers)
        return fail(REWL_EINVAL, "more than 4096 walkers: the static record buffer holds 4096 records");
    int dev = 0;
    HIP_TRY(hipStreamGetDevice(r->stream, &dev));
    double *buf = nullptr;
    st = scratch_on(dev, &buf);
    if (st != REWL_OK) return st;
    const size_t bytes = (size_t)d.nw * 8 * sizeof(double);
    HIP_TRY(rewl_gpu::launch_lipid_structure(d.spins, (size_t)d.Npad, (const unsigned char *)d.spins + d.lip_off_lip,
                                             (size_t)d.Npad, d.nw, d.nb, d.nmol, d.box, buf, r->stream));
    HIP_TRY(hipMemcpyAsync(out, buf, bytes, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return REWL_OK;
}

extern "C" int rewl_structure(rewl_t *r, double *out) {
    if (!r || !out) return fail(REWL_EINVAL, "null argument");
    const rewl_gpu::DevState &d = r->st;
    if (d.model != rewl_gpu::kModelLipid3D) return fail(REWL_EINVAL, "not a run of the lipid model");
    int st = check_structure_args(d.nw, d.nb, d.nmol, d.box);
    if (st != REWL_OK) return st;
    double *dev = nullptr;
    const size_t bytes = (size_t)d.nw * 8 * sizeof(double);
    HIP_TRY(hipMalloc((void **)&dev, bytes));
    hipError_t e = rewl_gpu::launch_lipid_structure(d.spins, (size_t)d.Npad, (const unsigned char *)d.spins + d.lip_off_lip,
                                                    (size_t)d.Npad, d.nw, d.nb, d.nmol, d.box, dev, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dev, bytes, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(REWL_EDEVICE, std::string("structure kernel: ") + hipGetErrorString(e));
    return REWL_OK;
}
