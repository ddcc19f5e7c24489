// Allocation-free evaluation (lss_eval_noalloc): the evaluation of lss_eval
// with every per-call device buffer (target copies, sort keys and workspace,
// tile lists, the device-side target count) carved out of one static device
// array instead of the context's grow-only allocations.  The kernels are
// those of lss_eval, launched in the same order on the same inputs, so the
// results are the same bit for bit.
//
// The array lives in the code object: each device that loads the library
// holds its own copy until the process ends.  Its device address is looked up
// once per device with hipGetSymbolAddress (lss_create does it for the
// context's device); host code uses only that address, never the array's
// name.  Every call on one device shares the array, so calls that overlap on
// one device (two contexts on two streams, say) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lss_internal.h"

namespace lss {
namespace {

constexpr size_t kScratchBytes = (size_t)48 << 20;     // 48 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};
std::string g_scratch_err[kMaxDevices];

// word 0: the target count (int32); word 2-3: mesh-id error count (u64)
__global__ void k_noalloc_words(int32_t *w, int32_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        w[0] = n;
        w[1] = 0;
        w[2] = 0;
        w[3] = 0;
    }
}

__global__ void k_noalloc_check_mesh(int64_t n, const int32_t *__restrict__ xm, int32_t nmesh,
                                     unsigned long long *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (xm[i] < 0 || xm[i] >= nmesh)) atomicAdd(bad, 1ull);
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte offsets of the per-call buffers for up to nmax targets.
struct Layout {
    size_t words, tx, ty, tz, tmesh, key, key2, perm, perm2, flag, pos, blocksum, tstart, tleaf, order, sort;
    size_t sort_bytes, total;
};

Layout layout_for(int64_t nmax) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    const size_t n = (size_t)nmax, n1 = n + 1;
    L.words = take(64);
    L.tx = take(8 * n);
    L.ty = take(8 * n);
    L.tz = take(8 * n);
    L.tmesh = take(4 * n);
    L.key = take(8 * n);
    L.key2 = take(8 * n);
    L.perm = take(4 * n);
    L.perm2 = take(4 * n);
    L.flag = take(4 * n1);
    L.pos = take(4 * n1);
    L.blocksum = take(4 * ((size_t)compact_blocks(nmax) + 2));
    L.tstart = take(4 * n1);
    L.tleaf = take(4 * n1);
    L.order = take(4 * n1);
    L.sort_bytes = sort_pairs_u64_tmp_bytes(nmax);
    L.sort = take(L.sort_bytes);
    L.total = o;
    return L;
}

}  // namespace

// Device address of the scratch array on `device` (the current device);
// looked up on the first call per device.  Null if the lookup failed; the
// message is then in *err.
void *noalloc_scratch(int device, std::string *err) {
    if (device < 0 || device >= kMaxDevices) {
        if (err) *err = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device] && g_scratch_err[device].empty()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        else
            g_scratch[device] = p;
    }
    if (!g_scratch[device] && err) *err = g_scratch_err[device];
    return g_scratch[device];
}

// lss_eval on device pointers with the per-call buffers in the scratch array.
void eval_noalloc(Ctx &c, const double *x, const int32_t *xm, int64_t n, double *phi, double *grad,
                  unsigned flags) {
    if (!(flags & LSS_PTR_DEVICE))
        throw Error{LSS_EINVAL, "lss_eval_noalloc: needs device pointers (LSS_PTR_DEVICE); host arrays would need "
                                "staging buffers"};
    if (n < 0) throw Error{LSS_EINVAL, "lss_eval_noalloc: n < 0"};
    if (n > LSS_NOALLOC_MAX_TARGETS)
        throw Error{LSS_EINVAL, "lss_eval_noalloc: n = " + std::to_string(n) + " exceeds LSS_NOALLOC_MAX_TARGETS (" +
                                    std::to_string((long long)LSS_NOALLOC_MAX_TARGETS) + "); use lss_eval"};
    if (n == 0) return;
    if (!x || !phi) throw Error{LSS_EINVAL, "lss_eval_noalloc: x and phi must be non-null"};
    if (c.nmesh > 1 && !xm) throw Error{LSS_EINVAL, "lss_eval_noalloc: x_mesh is required for a batch of meshes"};
    if (!c.built)
        throw Error{LSS_ESTATE, "lss_eval_noalloc: the context is not built (call lss_build after setting sources, "
                                "sigma and options; this entry point does not build)"};
    std::string err;
    unsigned char *base = static_cast<unsigned char *>(noalloc_scratch(c.device, &err));
    if (!base) throw Error{LSS_EHIP, "lss_eval_noalloc: " + err};
    const Layout L = layout_for(LSS_NOALLOC_MAX_TARGETS);
    if (L.total > kScratchBytes)
        throw Error{LSS_EHIP, "lss_eval_noalloc: scratch layout (" + std::to_string(L.total) +
                                  " bytes) exceeds the static array"};
    int32_t *words = reinterpret_cast<int32_t *>(base + L.words);
    hipLaunchKernelGGL(k_noalloc_words, dim3(1), dim3(64), 0, c.stream, words, (int32_t)n);
    LSS_CHECK_LAUNCH("k_noalloc_words");
    const int32_t *dxm = c.nmesh > 1 ? xm : nullptr;
    if (dxm) {      // mesh ids index per-mesh tables in every kernel: checked first (the call waits for it)
        unsigned long long *bad = reinterpret_cast<unsigned long long *>(words + 2);
        hipLaunchKernelGGL(k_noalloc_check_mesh, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c.stream, n, dxm,
                           c.nmesh, bad);
        LSS_CHECK_LAUNCH("k_noalloc_check_mesh");
        unsigned long long nb = 0;
        LSS_HIP(hipMemcpyAsync(&nb, bad, sizeof(nb), hipMemcpyDeviceToHost, c.stream));
        LSS_HIP(hipStreamSynchronize(c.stream));
        if (nb) throw Error{LSS_EINVAL, "lss_eval_noalloc: x_mesh values outside [0, nmesh)"};
    }
    EvalBufs b;
    b.tx = reinterpret_cast<double *>(base + L.tx);
    b.ty = reinterpret_cast<double *>(base + L.ty);
    b.tz = reinterpret_cast<double *>(base + L.tz);
    b.tmesh = reinterpret_cast<int32_t *>(base + L.tmesh);
    b.key = reinterpret_cast<uint64_t *>(base + L.key);
    b.key2 = reinterpret_cast<uint64_t *>(base + L.key2);
    b.perm = reinterpret_cast<int32_t *>(base + L.perm);
    b.perm2 = reinterpret_cast<int32_t *>(base + L.perm2);
    b.flag = reinterpret_cast<int32_t *>(base + L.flag);
    b.pos = reinterpret_cast<int32_t *>(base + L.pos);
    b.blocksum = reinterpret_cast<int32_t *>(base + L.blocksum);
    b.tstart = reinterpret_cast<int32_t *>(base + L.tstart);
    b.tleaf = reinterpret_cast<int32_t *>(base + L.tleaf);
    b.ntiles = words + 4;
    b.order = reinterpret_cast<int32_t *>(base + L.order);
    b.sort_tmp = base + L.sort;
    b.sort_bytes = L.sort_bytes;
    b.pairs = nullptr;                  // no statistics: lss_get_stats keeps the last lss_eval's
    b.n_dev = words;
    if (c.opt.far_field == LSS_FAR_FMM) {
        launch_soa(c, x, n, b.tx, b.ty, b.tz);
        if (dxm) LSS_HIP(hipMemcpyAsync(b.tmesh, dxm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
        eval_fmm_bufs(c, b, n, phi, grad);
    } else {
        eval_direct_bufs(c, b, x, dxm, n, phi, grad);
    }
}

}  // namespace lss
