// C-ABI layer of libpauli: argument validation, algorithm/tile dispatch,
// per-thread error messages, the tune table and the batched graph cache.
// Every check runs before any HIP call, so invalid requests fail without a
// device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pauli.h"
#include "common.hpp"
#include "internal.hpp"

using namespace pauli;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(PAULI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int N_MAX = 16;
constexpr int N_MAX_BATCHED = 12;

size_t elem_bytes(int dtype) { return dtype == PAULI_C128 ? 16 : 8; }

bool valid_dtype(int d) { return d == PAULI_C64 || d == PAULI_C128; }
bool valid_algo(int a) {
    return a == PAULI_ALGO_FP64_GRAY || a == PAULI_ALGO_FP32 || a == PAULI_ALGO_SPLIT_BF16 || a == PAULI_ALGO_FWHT ||
           a == PAULI_ALGO_SPLIT_FP16 || a == PAULI_ALGO_FWHT_F32 || a == PAULI_ALGO_SPLIT_I8;
}

// Fixed-point int8 algorithm: forward decomposition only, one tile shape.
bool is_i8(int a) { return a == PAULI_ALGO_SPLIT_I8; }

// Fast Walsh-Hadamard algorithms (binary64 or binary32 intermediate).
bool is_fwht(int a) { return a == PAULI_ALGO_FWHT || a == PAULI_ALGO_FWHT_F32; }

// Matrix-core algorithms (packed operand, tile shapes, separate passes).
bool is_mfma(int a) { return a == PAULI_ALGO_FP32 || a == PAULI_ALGO_SPLIT_BF16 || a == PAULI_ALGO_SPLIT_FP16; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

pauli_opts resolve(const pauli_opts* o) {
    pauli_opts r;
    pauli_opts_default(&r);
    if (o) r = *o;
    return r;
}

// Tune tables: (algo, N) -> tile id chosen by pauli_autotune, and (planes,
// sorted N list) -> persistent tile shape chosen by pauli_autotune_batched.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tune;
std::map<std::pair<int, std::vector<int>>, int> g_btile;
bool g_tune_loaded = false;

// Largest batch a tune-file line may describe.
constexpr size_t TUNE_MAX_COUNT = (size_t)1 << 20;

// The file named by PAULI_TUNE_CACHE, one entry per line:
//   "algo N tile"                      single matrices
//   "B planes tile c_1 c_2 ... c_12"   a batch with c_n matrices of order n
// Lines that do not parse are ignored.
void load_tune_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("PAULI_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        if (!line.empty() && line[0] == 'B') {
            std::string tag;
            int planes = 0, tile = 0;
            if (!(in >> tag >> planes >> tile)) continue;
            std::vector<int> ns;
            bool ok = true;
            for (int n = 1; n <= N_MAX_BATCHED && ok; ++n) {
                int c = -1;
                // a count no batch can have marks a damaged line (and would
                // otherwise make this loop allocate without bound)
                ok = (bool)(in >> c) && c >= 0 && ns.size() + (size_t)c <= TUNE_MAX_COUNT;
                if (ok) ns.insert(ns.end(), (size_t)c, n);
            }
            if (ok && !ns.empty()) g_btile[{planes, ns}] = tile;
        } else {
            int a, n, t;
            if (in >> a >> n >> t) g_tune[{a, n}] = t;
        }
    }
}

// Rewrite the tune file (if PAULI_TUNE_CACHE is set) with both tables.
bool save_tune_cache_locked() {
    const char* path = getenv("PAULI_TUNE_CACHE");
    if (!path) return true;
    FILE* f = fopen(path, "w");
    if (!f) return false;
    for (auto& kv : g_tune) fprintf(f, "%d %d %d\n", kv.first.first, kv.first.second, kv.second);
    for (auto& kv : g_btile) {
        int counts[N_MAX_BATCHED + 1] = {0};
        for (int n : kv.first.second) counts[n]++;
        fprintf(f, "B %d %d", kv.first.first, kv.second);
        for (int n = 1; n <= N_MAX_BATCHED; ++n) fprintf(f, " %d", counts[n]);
        fprintf(f, "\n");
    }
    fclose(f);
    return true;
}

int planes_of(int algo) {
    return algo == PAULI_ALGO_SPLIT_BF16 ? 3 : (algo == PAULI_ALGO_SPLIT_FP16 ? 2 : 1);
}

int pick_tile(int algo, int N, int forced) {
    if (!is_mfma(algo)) return 0;
    const int planes = planes_of(algo);
    if (forced > 0) return forced;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    auto it = g_tune.find({algo, N});
    if (it != g_tune.end() && mfma_tile_valid(planes, it->second, N)) return it->second;
    return mfma_default_tile(planes, N);
}

int check_common(const void* in, int N, int batch, const void* out, const pauli_opts& o,
                 const char* fn) {
    if (N < 0 || N > N_MAX) return fail(PAULI_EINVAL, "%s: N=%d outside [0, %d]", fn, N, N_MAX);
    if (batch < 1) return fail(PAULI_EINVAL, "%s: batch=%d must be >= 1", fn, batch);
    if (!in || !out) return fail(PAULI_EINVAL, "%s: NULL data pointer", fn);
    if (!valid_algo(o.algo)) return fail(PAULI_EINVAL, "%s: unknown algo %d", fn, o.algo);
    if (!valid_dtype(o.in_dtype) || !valid_dtype(o.out_dtype))
        return fail(PAULI_EINVAL, "%s: unknown dtype (in %d, out %d)", fn, o.in_dtype, o.out_dtype);
    if ((uintptr_t)in % 16) return fail(PAULI_EINVAL, "%s: input not aligned to 16 bytes", fn);
    if ((uintptr_t)out % 16) return fail(PAULI_EINVAL, "%s: output not aligned to 16 bytes", fn);
    const size_t count = ((size_t)1 << (2 * N)) * (size_t)batch;
    if (overlaps(in, count * elem_bytes(o.in_dtype), out, count * elem_bytes(o.out_dtype)))
        return fail(PAULI_EINVAL, "%s: input and output overlap", fn);
    if (o.tile < 0) return fail(PAULI_EINVAL, "%s: tile=%d must be >= 0", fn, o.tile);
    if (is_fwht(o.algo) && !fwht_supported(N))
        return fail(PAULI_EUNSUPPORTED, "%s: the FWHT algorithm covers %d <= N <= %d, not N=%d", fn, FWHT_N_MIN,
                    FWHT_N_MAX, N);
    if (o.workspace && o.algo != PAULI_ALGO_FP64_GRAY) {
        if ((uintptr_t)o.workspace % 256)
            return fail(PAULI_EINVAL, "%s: workspace must be 256-byte aligned", fn);
        if (overlaps(o.workspace, o.workspace_bytes, in, count * elem_bytes(o.in_dtype)) ||
            overlaps(o.workspace, o.workspace_bytes, out, count * elem_bytes(o.out_dtype)))
            return fail(PAULI_EINVAL, "%s: workspace overlaps input or output", fn);
    }
    if (o.tile > 1 && is_i8(o.algo))
        return fail(PAULI_EINVAL, "%s: tile %d not valid for algo %d (one tile shape)", fn, o.tile, o.algo);
    if (o.tile > 0 && is_mfma(o.algo) && !mfma_tile_valid(planes_of(o.algo), o.tile, N))
        return fail(PAULI_EINVAL, "%s: tile %d not valid for algo %d at N=%d", fn, o.tile, o.algo, N);
    return PAULI_OK;
}

// Library-owned stream-ordered pool per device for the packed operand when
// the caller passes no workspace; its release threshold keeps freed blocks
// for reuse by later calls instead of returning them at each synchronisation.
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;

hipError_t pool_for_current_device(hipMemPool_t* pool) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) {
        *pool = it->second;
        return hipSuccess;
    }
    hipMemPoolProps props;
    memset(&props, 0, sizeof props);
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    e = hipMemPoolCreate(pool, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = ~(uint64_t)0;
    e = hipMemPoolSetAttribute(*pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
        (void)hipMemPoolDestroy(*pool);   // not kept: the next call tries again
        return e;
    }
    g_pools[dev] = *pool;
    return hipSuccess;
}

// Tile for the Hermitian forward contraction: forced, else the tuned tile of
// the general path when it is a register-ring tile, else the default.
// The Hermitian contraction has its own defaults: the tune table holds tiles
// timed on the general contraction, whose work per tile differs.
int pick_tile_hermitian(int algo, int N, int forced) {
    if (forced > 0) return forced;
    return mfma_default_tile_hermitian(planes_of(algo), N);
}

int run(Dir dir, const void* in, int N, int batch, void* out, const pauli_opts& o, double scale,
        const char* fn, bool herm = false) {
    hipError_t e;
    hipStream_t s = (hipStream_t)o.stream;
    const bool in128 = o.in_dtype == PAULI_C128, out128 = o.out_dtype == PAULI_C128;
    if (o.algo == PAULI_ALGO_FP64_GRAY) {
        e = launch_gray(dir, in, in128, out, out128, N, batch, scale, s);
    } else if (is_fwht(o.algo)) {
        const bool narrow = o.algo == PAULI_ALGO_FWHT_F32;
        const size_t need = fwht_workspace_bytes(N, batch, narrow);
        void* ws = o.workspace;
        if (need == 0) {
            e = launch_fwht(dir, in, in128, out, out128, N, batch, scale, narrow, nullptr, s);
        } else if (ws) {
            if (o.workspace_bytes < need)
                return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need,
                            o.workspace_bytes);
            e = launch_fwht(dir, in, in128, out, out128, N, batch, scale, narrow, ws, s);
        } else {
            hipMemPool_t pool;
            if ((e = pool_for_current_device(&pool)) != hipSuccess) return hip_fail(e, fn);
            if ((e = hipMallocFromPoolAsync(&ws, need, pool, s)) != hipSuccess) return hip_fail(e, fn);
            e = launch_fwht(dir, in, in128, out, out128, N, batch, scale, narrow, ws, s);
            const hipError_t ef = hipFreeAsync(ws, s);
            if (e == hipSuccess) e = ef;
        }
    } else if (is_i8(o.algo)) {
        const size_t need = i8_workspace_bytes(N, batch);
        void* ws = o.workspace;
        if (ws) {
            if (o.workspace_bytes < need)
                return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need,
                            o.workspace_bytes);
            e = launch_i8(dir, in, in128, out, out128, N, batch, scale, ws, herm, s);
        } else {
            hipMemPool_t pool;
            if ((e = pool_for_current_device(&pool)) != hipSuccess) return hip_fail(e, fn);
            if ((e = hipMallocFromPoolAsync(&ws, need, pool, s)) != hipSuccess) return hip_fail(e, fn);
            e = launch_i8(dir, in, in128, out, out128, N, batch, scale, ws, herm, s);
            const hipError_t ef = hipFreeAsync(ws, s);
            if (e == hipSuccess) e = ef;
        }
    } else {
        const int planes = planes_of(o.algo);
        const int tile = herm ? pick_tile_hermitian(o.algo, N, o.tile) : pick_tile(o.algo, N, o.tile);
        const size_t need = mfma_workspace_bytes(planes, N, batch);
        auto launch = [&](void* w) {
            return herm ? launch_mfma_hermitian(planes, in, in128, out, out128, N, batch, scale, tile, w, s)
                        : launch_mfma(dir, planes, in, in128, out, out128, N, batch, scale, tile, w, s);
        };
        void* ws = o.workspace;
        if (ws) {
            if (o.workspace_bytes < need)
                return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need,
                            o.workspace_bytes);
            e = launch(ws);
        } else {
            hipMemPool_t pool;
            if ((e = pool_for_current_device(&pool)) != hipSuccess) return hip_fail(e, fn);
            if ((e = hipMallocFromPoolAsync(&ws, need, pool, s)) != hipSuccess) return hip_fail(e, fn);
            e = launch(ws);
            const hipError_t ef = hipFreeAsync(ws, s);
            if (e == hipSuccess) e = ef;
        }
    }
    if (e != hipSuccess) return hip_fail(e, fn);
    g_last_error.clear();
    return PAULI_OK;
}

// Fixed device scratch of pauli_decompose_noalloc: one copy per GPU, held
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not the device copy: kernels get the device address looked up once per
// device with hipGetSymbolAddress (with that device current) and kept here.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its copy

hipError_t scratch_for_current_device(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
    *ptr = p;
    return hipSuccess;
}

}  // namespace

extern "C" {

void pauli_opts_default(pauli_opts* o) {
    if (!o) return;
    o->algo = PAULI_ALGO_SPLIT_BF16;
    o->in_dtype = PAULI_C64;
    o->out_dtype = PAULI_C64;
    o->tile = 0;
    o->stream = nullptr;
    o->workspace = nullptr;
    o->workspace_bytes = 0;
}

int pauli_decompose(const void* G, int N, int batch, void* out, const pauli_opts* opts) {
    const pauli_opts o = resolve(opts);
    int st = check_common(G, N, batch, out, o, "pauli_decompose");
    if (st != PAULI_OK) return st;
    return run(FORWARD, G, N, batch, out, o, 1.0 / (double)(1u << N), "pauli_decompose");
}

int pauli_decompose_noalloc(const void* G, int N, int batch, void* out, const pauli_opts* opts) {
    const char* fn = "pauli_decompose_noalloc";
    pauli_opts o = resolve(opts);
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    int st = check_common(G, N, batch, out, o, fn);
    if (st != PAULI_OK) return st;
    size_t need = 0;
    if (is_fwht(o.algo)) need = fwht_workspace_bytes(N, batch, o.algo == PAULI_ALGO_FWHT_F32);
    else if (is_mfma(o.algo)) need = mfma_workspace_bytes(planes_of(o.algo), N, batch);
    else if (is_i8(o.algo)) need = i8_workspace_bytes(N, batch);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(PAULI_ENOMEM, "%s: algo %d at N=%d, batch %d needs %zu bytes of scratch; the fixed scratch holds %zu",
                    fn, o.algo, N, batch, need, NOALLOC_SCRATCH_BYTES);
    if (need > 0) {
        void* p = nullptr;
        const hipError_t e = scratch_for_current_device(&p);
        if (e != hipSuccess) return hip_fail(e, fn);
        o.workspace = p;
        o.workspace_bytes = NOALLOC_SCRATCH_BYTES;
    }
    return run(FORWARD, G, N, batch, out, o, 1.0 / (double)(1u << N), fn);
}

size_t pauli_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int pauli_decompose_hermitian(const void* G, int N, int batch, void* out, const pauli_opts* opts) {
    const char* fn = "pauli_decompose_hermitian";
    pauli_opts o = resolve(opts);
    if (valid_algo(o.algo) && !is_mfma(o.algo) && !is_i8(o.algo))
        return fail(PAULI_EUNSUPPORTED, "%s: algo %d has no Hermitian variant (the matrix-core algorithms have)",
                    fn, o.algo);
    const int forced = o.tile;
    o.tile = 0;   // the general tile check below does not apply; the Hermitian one does
    int st = check_common(G, N, batch, out, o, fn);
    if (st != PAULI_OK) return st;
    if (forced < 0) return fail(PAULI_EINVAL, "%s: tile=%d must be >= 0", fn, forced);
    if (forced > 0 && (is_i8(o.algo) ? forced != 1 : !mfma_tile_valid_hermitian(planes_of(o.algo), forced, N)))
        return fail(PAULI_EINVAL, "%s: tile %d not valid for the Hermitian variant of algo %d at N=%d", fn, forced,
                    o.algo, N);
    o.tile = forced;
    return run(FORWARD, G, N, batch, out, o, 1.0 / (double)(1u << N), fn, true);
}

int pauli_reconstruct(const void* c, int N, int batch, void* G, const pauli_opts* opts) {
    const pauli_opts o = resolve(opts);
    int st = check_common(c, N, batch, G, o, "pauli_reconstruct");
    if (st != PAULI_OK) return st;
    return run(ADJOINT, c, N, batch, G, o, 1.0, "pauli_reconstruct");
}

int pauli_decompose_backward(const void* grad_c, int N, int batch, void* grad_G,
                             const pauli_opts* opts) {
    const pauli_opts o = resolve(opts);
    int st = check_common(grad_c, N, batch, grad_G, o, "pauli_decompose_backward");
    if (st != PAULI_OK) return st;
    return run(ADJOINT, grad_c, N, batch, grad_G, o, 1.0 / (double)(1u << N),
               "pauli_decompose_backward");
}

static int stage_check(int N, int batch, int mode, const pauli_opts& o, const char* fn) {
    if (N < 0 || N > N_MAX) return fail(PAULI_EINVAL, "%s: N=%d outside [0, %d]", fn, N, N_MAX);
    if (batch < 1) return fail(PAULI_EINVAL, "%s: batch=%d must be >= 1", fn, batch);
    if (mode < 0 || mode > 3) return fail(PAULI_EINVAL, "%s: mode %d not in {0, 1, 2, 3}", fn, mode);
    if (!is_mfma(o.algo) && !is_i8(o.algo))
        return fail(PAULI_EUNSUPPORTED, "%s: algo %d has no separate passes", fn, o.algo);
    if (!valid_dtype(o.in_dtype) || !valid_dtype(o.out_dtype))
        return fail(PAULI_EINVAL, "%s: unknown dtype (in %d, out %d)", fn, o.in_dtype, o.out_dtype);
    const size_t need = is_i8(o.algo) ? i8_workspace_bytes(N, batch) : mfma_workspace_bytes(planes_of(o.algo), N, batch);
    if (!o.workspace || o.workspace_bytes < need)
        return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need,
                    o.workspace ? o.workspace_bytes : (size_t)0);
    if ((uintptr_t)o.workspace % 256) return fail(PAULI_EINVAL, "%s: workspace must be 256-byte aligned", fn);
    if (is_i8(o.algo)) {
        if (o.tile < 0 || o.tile > 1) return fail(PAULI_EINVAL, "%s: tile %d not valid at N=%d", fn, o.tile, N);
    } else if (o.tile < 0 || (o.tile > 0 && !(mode == 3 ? mfma_tile_valid_hermitian(planes_of(o.algo), o.tile, N)
                                                        : mfma_tile_valid(planes_of(o.algo), o.tile, N))))
        return fail(PAULI_EINVAL, "%s: tile %d not valid at N=%d", fn, o.tile, N);
    return PAULI_OK;
}

int pauli_pack(const void* in, int N, int batch, int mode, const pauli_opts* opts) {
    const char* fn = "pauli_pack";
    const pauli_opts o = resolve(opts);
    int st = stage_check(N, batch, mode, o, fn);
    if (st != PAULI_OK) return st;
    if (!in) return fail(PAULI_EINVAL, "%s: NULL input", fn);
    if ((uintptr_t)in % 16) return fail(PAULI_EINVAL, "%s: input not aligned to 16 bytes", fn);
    const size_t bytes = ((size_t)1 << (2 * N)) * (size_t)batch * elem_bytes(o.in_dtype);
    if (overlaps(in, bytes, o.workspace, o.workspace_bytes))
        return fail(PAULI_EINVAL, "%s: workspace overlaps the input", fn);
    const hipError_t e =
        is_i8(o.algo) ? launch_i8_pack(in, o.in_dtype == PAULI_C128, N, batch, o.workspace,
                                       mode == 1 || mode == 2 ? ADJOINT : FORWARD, mode == 3, (hipStream_t)o.stream)
        : mode == 3 ? launch_mfma_pack_hermitian(planes_of(o.algo), in, o.in_dtype == PAULI_C128, N, batch, o.workspace,
                                               (hipStream_t)o.stream)
                  : launch_mfma_pack(mode == 0 ? FORWARD : ADJOINT, planes_of(o.algo), in, o.in_dtype == PAULI_C128, N,
                                     batch, o.workspace, (hipStream_t)o.stream);
    if (e != hipSuccess) return hip_fail(e, fn);
    g_last_error.clear();
    return PAULI_OK;
}

int pauli_contract(int N, int batch, int mode, void* out, const pauli_opts* opts) {
    const char* fn = "pauli_contract";
    const pauli_opts o = resolve(opts);
    int st = stage_check(N, batch, mode, o, fn);
    if (st != PAULI_OK) return st;
    if (!out) return fail(PAULI_EINVAL, "%s: NULL output", fn);
    if ((uintptr_t)out % 16) return fail(PAULI_EINVAL, "%s: output not aligned to 16 bytes", fn);
    const size_t bytes = ((size_t)1 << (2 * N)) * (size_t)batch * elem_bytes(o.out_dtype);
    if (overlaps(out, bytes, o.workspace, o.workspace_bytes))
        return fail(PAULI_EINVAL, "%s: workspace overlaps the output", fn);
    const double scale = mode == 1 ? 1.0 : 1.0 / (double)(1u << N);
    const hipError_t e =
        is_i8(o.algo) ? launch_i8_contract(o.workspace, out, o.out_dtype == PAULI_C128, N, batch, scale,
                                           mode == 1 || mode == 2 ? ADJOINT : FORWARD, mode == 3, (hipStream_t)o.stream)
        : mode == 3 ? launch_mfma_contract_hermitian(planes_of(o.algo), o.workspace, out, o.out_dtype == PAULI_C128, N,
                                                   batch, scale, pick_tile_hermitian(o.algo, N, o.tile),
                                                   (hipStream_t)o.stream)
                  : launch_mfma_contract(mode == 0 ? FORWARD : ADJOINT, planes_of(o.algo), o.workspace, out,
                                         o.out_dtype == PAULI_C128, N, batch, scale, pick_tile(o.algo, N, o.tile),
                                         (hipStream_t)o.stream);
    if (e != hipSuccess) return hip_fail(e, fn);
    g_last_error.clear();
    return PAULI_OK;
}

size_t pauli_workspace_bytes(int algo, int N, int batch) {
    if (!valid_algo(algo) || N < 0 || N > N_MAX || batch < 1) return 0;
    if (algo == PAULI_ALGO_FP64_GRAY) return 0;
    if (is_fwht(algo)) return fwht_supported(N) ? fwht_workspace_bytes(N, batch, algo == PAULI_ALGO_FWHT_F32) : 0;
    if (is_i8(algo)) return i8_workspace_bytes(N, batch);
    return mfma_workspace_bytes(planes_of(algo), N, batch);
}

int pauli_tile_count(int algo) {
    if (algo == PAULI_ALGO_FP64_GRAY || is_fwht(algo) || is_i8(algo)) return 1;
    if (!valid_algo(algo)) return 0;
    return mfma_tile_count(planes_of(algo));
}

int pauli_tile_valid(int algo, int tile, int N) {
    if (algo == PAULI_ALGO_FP64_GRAY) return tile == 1 && N >= 0 && N <= N_MAX ? 1 : 0;
    if (is_fwht(algo)) return tile == 1 && fwht_supported(N) ? 1 : 0;
    if (is_i8(algo)) return tile == 1 && N >= 0 && N <= N_MAX ? 1 : 0;
    if (!valid_algo(algo) || N < 0 || N > N_MAX) return 0;
    return mfma_tile_valid(planes_of(algo), tile, N) ? 1 : 0;
}

int pauli_tile_valid_hermitian(int algo, int tile, int N) {
    if (is_i8(algo)) return tile == 1 && N >= 0 && N <= N_MAX ? 1 : 0;
    if (!is_mfma(algo) || N < 0 || N > N_MAX) return 0;
    return mfma_tile_valid_hermitian(planes_of(algo), tile, N) ? 1 : 0;
}

int pauli_tile_selected(int algo, int N) {
    if (!valid_algo(algo) || N < 0 || N > N_MAX) return 0;
    return pick_tile(algo, N, 0);
}

int pauli_tile_selected_hermitian(int algo, int N) {
    if (!is_mfma(algo) || N < 0 || N > N_MAX) return 0;
    return pick_tile_hermitian(algo, N, 0);
}

const char* pauli_last_error(void) { return g_last_error.c_str(); }

int pauli_version(void) { return 1; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Uneven batch: batched pack + persistent contraction behind a cached graph.
// Workspace layout: [descriptor table, pack and tile slot tables | counter |
// (two-plane split: prescale exponents per slot | partial maxima per pack
// tile) | packed operands]; the tile slot table is sized for the tile shape
// with the most tiles, so one workspace size serves every shape.
// ---------------------------------------------------------------------------
namespace {

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

struct BatchLayout {
    std::vector<int> order;        // matrix index of every descriptor slot (LPT: larger N first)
    std::vector<size_t> ws_off;    // per slot
    std::vector<uint32_t> pack0;   // per slot
    std::vector<uint32_t> tile0;   // per slot
    uint32_t pack_total = 0, tile_total = 0;
    size_t items_bytes = 0, table_bytes = 0, counter_off = 0, packed_off = 0, total_bytes = 0;
    size_t pe_off = 0, partial_off = 0;   // two-plane split: prescale exponents, partial maxima
    std::vector<uint32_t> pack_slot;   // slot of every pack tile
    std::vector<uint32_t> tile_slot;   // slot of every output tile
    std::vector<uint32_t> queues;      // [nq | nq + 1 offsets | output tile ids], see launch_batched
    size_t staged_bytes = 0;           // descriptors + pack slots + tile slots + queues
};

// Deal the flip-mask slabs of the batch (every row block of a slab together)
// to nq queues, each slab to the least loaded queue, in slot order (largest
// matrices first).  A slab's estimated cost is its D x D multiply-adds per
// row-block tile plus a fixed per-tile overhead.
std::vector<uint32_t> batch_queues(const BatchLayout& L, const int* N, int btile) {
    const uint32_t nq = std::min<uint32_t>(MAX_QUEUES, L.tile_total);
    std::vector<std::vector<uint32_t>> q(nq);
    std::vector<double> load(nq, 0.0);
    for (size_t slot = 0; slot < L.order.size(); ++slot) {
        const int n = N[L.order[slot]];
        const uint32_t Dp = n < 5 ? 32u : (1u << n), nXB = Dp / 32u;
        const uint32_t nMB = batched_output_tiles(btile, n) / nXB;
        const double cost = (double)nMB * ((double)Dp * (double)Dp + 16384.0);
        for (uint32_t xb = 0; xb < nXB; ++xb) {
            const uint32_t k = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
            for (uint32_t mb = 0; mb < nMB; ++mb) q[k].push_back(L.tile0[slot] + xb * nMB + mb);
            load[k] += cost;
        }
    }
    std::vector<uint32_t> out{nq};
    uint32_t off = 0;
    for (uint32_t k = 0; k < nq; ++k) {
        out.push_back(off);
        off += (uint32_t)q[k].size();
    }
    out.push_back(off);
    for (uint32_t k = 0; k < nq; ++k) out.insert(out.end(), q[k].begin(), q[k].end());
    return out;
}

BatchLayout batch_layout(int count, const int* N, int planes, int btile) {
    BatchLayout L;
    L.order.resize(count);
    for (int k = 0; k < count; ++k) L.order[k] = k;
    std::stable_sort(L.order.begin(), L.order.end(), [&](int a, int b) { return N[a] > N[b]; });
    size_t off = 0, max_tiles = 0;
    for (int slot = 0; slot < count; ++slot) {
        const int n = N[L.order[slot]];
        L.ws_off.push_back(off);
        L.pack0.push_back(L.pack_total);
        L.tile0.push_back(L.tile_total);
        off += round256(batched_packed_bytes(planes, n));
        L.pack_slot.insert(L.pack_slot.end(), batched_pack_tiles(n), (uint32_t)slot);
        L.pack_total += batched_pack_tiles(n);
        const uint32_t tiles = batched_output_tiles(btile, n);
        L.tile_slot.insert(L.tile_slot.end(), tiles, (uint32_t)slot);
        L.tile_total += tiles;
        uint32_t most = 0;
        for (int b = 1; b <= batched_tile_count(); ++b) most = std::max(most, batched_output_tiles(b, n));
        max_tiles += most;
    }
    L.items_bytes = sizeof(BatchItem) * (size_t)count;
    L.queues = batch_queues(L, N, btile);
    L.staged_bytes = L.items_bytes + sizeof(uint32_t) * ((size_t)L.pack_total + L.tile_total + L.queues.size());
    // descriptors, pack slots, output slots and queues (room for the tile
    // shape with the most tiles)
    L.table_bytes =
        round256(L.items_bytes + sizeof(uint32_t) * ((size_t)L.pack_total + 2 * max_tiles + 2 + MAX_QUEUES));
    L.counter_off = L.table_bytes;
    size_t next = L.counter_off + 256;
    if (planes == 2) {
        L.pe_off = next;
        L.partial_off = L.pe_off + round256(sizeof(int) * (size_t)count);
        next = L.partial_off + round256(sizeof(float) * (size_t)L.pack_total);
    }
    L.packed_off = next;
    L.total_bytes = L.packed_off + off;
    return L;
}

struct GraphKey {
    hipStream_t stream;
    void* workspace;
    int planes, btile;
    std::vector<int> ns;
    bool operator<(const GraphKey& o) const {
        return std::tie(stream, workspace, planes, btile, ns) < std::tie(o.stream, o.workspace, o.planes, o.btile, o.ns);
    }
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    BatchLayout layout;
    unsigned char* pinned = nullptr;   // host staging of the descriptor and tile slot tables
    hipEvent_t copied = nullptr;   // the staging may be rewritten once this has fired
    hipEvent_t done = nullptr;     // the last replay has finished once this has fired
    uint64_t last_use = 0;
};

// At most this many captured batches are kept; the least recently used one
// makes room for a new one (after its last replay and staging copy finish).
constexpr size_t MAX_GRAPHS = 64;
std::mutex g_graph_mu;
std::map<GraphKey, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;

void release_entry(GraphEntry& g) {
    if (g.done) (void)hipEventSynchronize(g.done);
    if (g.copied) (void)hipEventSynchronize(g.copied);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.pinned) (void)hipHostFree(g.pinned);
    if (g.copied) (void)hipEventDestroy(g.copied);
    if (g.done) (void)hipEventDestroy(g.done);
    g = GraphEntry{};
}

void evict_lru_locked() {
    auto victim = g_graphs.end();
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
        if (victim == g_graphs.end() || it->second.last_use < victim->second.last_use) victim = it;
    if (victim == g_graphs.end()) return;
    release_entry(victim->second);
    g_graphs.erase(victim);
}

int validate_batch(int count, const void* const* G, const int* N, void* const* out, const pauli_opts& o,
                   const char* fn) {
    if (count < 1) return fail(PAULI_EINVAL, "%s: count=%d must be >= 1", fn, count);
    if (!G || !N || !out) return fail(PAULI_EINVAL, "%s: NULL array", fn);
    if (!is_mfma(o.algo))
        return fail(PAULI_EUNSUPPORTED, "%s: algo %d not available batched (SPLIT_BF16, SPLIT_FP16 or FP32)", fn,
                    o.algo);
    if (o.in_dtype != PAULI_C64 || o.out_dtype != PAULI_C64)
        return fail(PAULI_EUNSUPPORTED, "%s: only C64 input and output", fn);
    if (o.tile < 0 || o.tile > batched_tile_count())
        return fail(PAULI_EINVAL, "%s: tile %d outside [0, %d]", fn, o.tile, batched_tile_count());
    if (o.tile > 0 && !batched_tile_valid(planes_of(o.algo), o.tile))
        return fail(PAULI_EINVAL, "%s: tile %d is not available for algo %d", fn, o.tile, o.algo);
    for (int k = 0; k < count; ++k) {
        if (N[k] < 1 || N[k] > N_MAX_BATCHED)
            return fail(PAULI_EINVAL, "%s: N[%d]=%d outside [1, %d]", fn, k, N[k], N_MAX_BATCHED);
        if (!G[k] || !out[k]) return fail(PAULI_EINVAL, "%s: NULL pointer for matrix %d", fn, k);
        if ((uintptr_t)G[k] % 16 || (uintptr_t)out[k] % 16)
            return fail(PAULI_EINVAL, "%s: matrix %d not 16-byte aligned", fn, k);
        const size_t bytes = ((size_t)1 << (2 * N[k])) * 8;
        if (overlaps(G[k], bytes, out[k], bytes))
            return fail(PAULI_EINVAL, "%s: input and output of matrix %d overlap", fn, k);
    }
    return PAULI_OK;
}

int tuned_btile(int planes, int count, const int* N) {
    std::vector<int> ns(N, N + count);
    std::sort(ns.begin(), ns.end());
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    auto it = g_btile.find({planes, ns});
    // a cached shape that is out of range or not built for these planes (a
    // hand-edited or stale file) falls back to the default shape
    if (it == g_btile.end() || !batched_tile_valid(planes, it->second)) return batched_default_tile(planes);
    return it->second;
}

int run_batched(int count, const void* const* G, const int* N, void* const* out, const pauli_opts& o, int btile,
                const char* fn) {
    const int planes = planes_of(o.algo);
    hipStream_t s = (hipStream_t)o.stream;
    GraphKey key{s, o.workspace, planes, btile, std::vector<int>(N, N + count)};
    std::lock_guard<std::mutex> lk(g_graph_mu);
    // a replay reuses the layout its graph was built with (same key, same layout)
    auto found = g_graphs.find(key);
    BatchLayout fresh;
    if (found == g_graphs.end() || !found->second.exec) fresh = batch_layout(count, N, planes, btile);
    const BatchLayout& probe = (found != g_graphs.end() && found->second.exec) ? found->second.layout : fresh;
    if (!o.workspace || o.workspace_bytes < probe.total_bytes)
        return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, probe.total_bytes,
                    o.workspace ? o.workspace_bytes : (size_t)0);
    if ((uintptr_t)o.workspace % 256) return fail(PAULI_EINVAL, "%s: workspace must be 256-byte aligned", fn);
    for (int k = 0; k < count; ++k) {
        const size_t bytes = ((size_t)1 << (2 * N[k])) * 8;
        if (overlaps(o.workspace, probe.total_bytes, G[k], bytes) ||
            overlaps(o.workspace, probe.total_bytes, out[k], bytes))
            return fail(PAULI_EINVAL, "%s: workspace overlaps matrix %d", fn, k);
    }
    unsigned char* ws = (unsigned char*)o.workspace;
    BatchItem* items_dev = (BatchItem*)ws;
    const uint32_t* pack_slot_dev = (const uint32_t*)(ws + probe.items_bytes);
    const uint32_t* tile_slot_dev = pack_slot_dev + probe.pack_total;
    const uint32_t* queues_dev = tile_slot_dev + probe.tile_total;
    const size_t staged = probe.staged_bytes;
    unsigned int* counter_dev = (unsigned int*)(ws + probe.counter_off);
    unsigned char* packed = ws + probe.packed_off;
    if (found == g_graphs.end() && g_graphs.size() >= MAX_GRAPHS) evict_lru_locked();
    GraphEntry& ge = found != g_graphs.end() ? found->second : g_graphs[key];
    ge.last_use = ++g_graph_clock;
    hipError_t e;
    if (!ge.exec) {
        ge.layout = probe;
        auto discard = [&](hipError_t err) {   // leave no half-built entry behind
            release_entry(ge);
            g_graphs.erase(key);
            return hip_fail(err, fn);
        };
        if ((e = hipHostMalloc((void**)&ge.pinned, staged)) != hipSuccess) return discard(e);
        memcpy(ge.pinned + probe.items_bytes, probe.pack_slot.data(), sizeof(uint32_t) * probe.pack_total);
        memcpy(ge.pinned + probe.items_bytes + sizeof(uint32_t) * probe.pack_total, probe.tile_slot.data(),
               sizeof(uint32_t) * probe.tile_total);
        memcpy(ge.pinned + probe.items_bytes + sizeof(uint32_t) * ((size_t)probe.pack_total + probe.tile_total),
               probe.queues.data(), sizeof(uint32_t) * probe.queues.size());
        if ((e = hipEventCreateWithFlags(&ge.copied, hipEventDisableTiming)) != hipSuccess) return discard(e);
        if ((e = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming)) != hipSuccess) return discard(e);
        // Capture on a private stream: batched pack (which zeroes the queue counters), persistent contraction.
        hipStream_t cap;
        if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return discard(e);
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            int* pe_dev = planes == 2 ? (int*)(ws + probe.pe_off) : nullptr;
            float* partial_dev = planes == 2 ? (float*)(ws + probe.partial_off) : nullptr;
            const hipError_t le = launch_batched(planes, btile, items_dev, pack_slot_dev, tile_slot_dev, queues_dev,
                                                 (uint32_t)count, probe.pack_total, probe.tile_total, packed,
                                                 counter_dev, pe_dev, partial_dev, cap);
            e = hipStreamEndCapture(cap, &graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) {
            ge.exec = nullptr;
            return discard(e);
        }
    }
    // Refresh the descriptor table: pointers may differ between calls.
    if ((e = hipEventSynchronize(ge.copied)) != hipSuccess) return hip_fail(e, fn);
    const BatchLayout& L = ge.layout;
    BatchItem* items_host = (BatchItem*)ge.pinned;
    for (int slot = 0; slot < count; ++slot) {
        const int k = L.order[slot];
        items_host[slot].in = G[k];
        items_host[slot].out = out[k];
        items_host[slot].ws_off = L.ws_off[slot];
        items_host[slot].n = N[k];
        items_host[slot].pack0 = L.pack0[slot];
        items_host[slot].tile0 = L.tile0[slot];
    }
    // both tables every call: another batch may have used this workspace since
    if ((e = hipMemcpyAsync(items_dev, ge.pinned, staged, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, fn);
    if ((e = hipEventRecord(ge.copied, s)) != hipSuccess) return hip_fail(e, fn);
    if ((e = hipGraphLaunch(ge.exec, s)) != hipSuccess) return hip_fail(e, fn);
    if ((e = hipEventRecord(ge.done, s)) != hipSuccess) return hip_fail(e, fn);
    g_last_error.clear();
    return PAULI_OK;
}

}  // namespace

extern "C" size_t pauli_batched_workspace_bytes(int count, const int* N, int algo) {
    if (count < 1 || !N || !is_mfma(algo)) return 0;
    for (int k = 0; k < count; ++k)
        if (N[k] < 1 || N[k] > N_MAX_BATCHED) return 0;
    return batch_layout(count, N, planes_of(algo), 1).total_bytes;
}

extern "C" int pauli_decompose_batched(int count, const void* const* G, const int* N, void* const* out,
                                       const pauli_opts* opts) {
    const char* fn = "pauli_decompose_batched";
    const pauli_opts o = resolve(opts);
    int st = validate_batch(count, G, N, out, o, fn);
    if (st != PAULI_OK) return st;
    const int btile = o.tile > 0 ? o.tile : tuned_btile(planes_of(o.algo), count, N);
    return run_batched(count, G, N, out, o, btile, fn);
}

extern "C" int pauli_autotune_batched(int count, const void* const* G, const int* N, void* const* out,
                                      const pauli_opts* opts) {
    const char* fn = "pauli_autotune_batched";
    const pauli_opts o = resolve(opts);
    int st = validate_batch(count, G, N, out, o, fn);
    if (st != PAULI_OK) return st;
    const int planes = planes_of(o.algo);
    hipStream_t s = (hipStream_t)o.stream;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int best = batched_default_tile(planes);
    float best_ms = 1e30f;
    for (int t = 1; t <= batched_tile_count() && e == hipSuccess; ++t) {
        if (!batched_tile_valid(planes, t)) continue;
        if ((st = run_batched(count, G, N, out, o, t, fn)) != PAULI_OK) break;   // warm-up + capture
        if ((e = hipEventRecord(a, s)) != hipSuccess) break;
        for (int r = 0; r < 5 && st == PAULI_OK; ++r) st = run_batched(count, G, N, out, o, t, fn);
        if (st != PAULI_OK) break;
        if ((e = hipEventRecord(b, s)) != hipSuccess) break;
        if ((e = hipEventSynchronize(b)) != hipSuccess) break;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (st != PAULI_OK) return st;
    if (e != hipSuccess) return hip_fail(e, fn);
    std::vector<int> ns(N, N + count);
    std::sort(ns.begin(), ns.end());
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_cache_locked();
        g_btile[{planes, ns}] = best;
        if (!save_tune_cache_locked())
            return fail(PAULI_EINVAL, "%s: cannot write %s", fn, getenv("PAULI_TUNE_CACHE"));
    }
    g_last_error.clear();
    return PAULI_OK;
}

extern "C" int pauli_batched_tile_count(void) { return batched_tile_count(); }

extern "C" int pauli_batched_tile_valid(int algo, int tile) {
    if (!is_mfma(algo)) return 0;
    return batched_tile_valid(planes_of(algo), tile) ? 1 : 0;
}

extern "C" int pauli_batched_tile_selected(int count, const int* N, int algo) {
    if (count < 1 || !N || !is_mfma(algo)) return 0;
    return tuned_btile(planes_of(algo), count, N);
}

// ---------------------------------------------------------------------------
// Autotuner: time each tile id per N on scratch matrices, keep the fastest.
// ---------------------------------------------------------------------------
namespace {

// 32-bit integer mixer (C. Wellons' "lowbias32" constants).
__device__ inline uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Autotuner input: a fixed pseudo-random complex64 matrix, each component
// uniform on [-1, 1) from the hash of its position.
__global__ __launch_bounds__(256) void tune_fill_kernel(float2* __restrict__ p, size_t n) {
    const float k = 1.0f / 2147483648.0f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const uint32_t h = mix32((uint32_t)(2 * i)), g = mix32((uint32_t)(2 * i + 1));
        p[i] = make_float2((float)(int32_t)h * k, (float)(int32_t)g * k);
    }
}

}  // namespace

extern "C" int pauli_autotune(int N_min, int N_max, const pauli_opts* opts) {
    const char* fn = "pauli_autotune";
    pauli_opts o = resolve(opts);
    if (!is_mfma(o.algo)) return fail(PAULI_EUNSUPPORTED, "%s: algo %d has no tile choice", fn, o.algo);
    if (N_min < 1 || N_max > N_MAX || N_min > N_max)
        return fail(PAULI_EINVAL, "%s: bad range [%d, %d]", fn, N_min, N_max);
    const int planes = planes_of(o.algo);
    hipStream_t s = (hipStream_t)o.stream;
    hipError_t e;
    for (int N = N_min; N <= N_max; ++N) {
        const size_t elems = (size_t)1 << (2 * N);
        void *in = nullptr, *out = nullptr, *ws = nullptr;
        if ((e = hipMalloc(&in, elems * 8)) != hipSuccess) return hip_fail(e, fn);
        if ((e = hipMalloc(&out, elems * 8)) != hipSuccess) {
            (void)hipFree(in);
            return hip_fail(e, fn);
        }
        if ((e = hipMalloc(&ws, mfma_workspace_bytes(planes, N, 1))) != hipSuccess) {
            (void)hipFree(in);
            (void)hipFree(out);
            return hip_fail(e, fn);
        }
        // operands like real data: zero operands draw less matrix-core power,
        // and the clock is power-limited, so a ranking taken on zeros may not hold
        hipEvent_t a = nullptr, b = nullptr;
        hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, s, (float2*)in, elems);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        int best = 0;
        float best_ms = 1e30f;
        const int ntiles = mfma_tile_count(planes);
        const int reps = N >= 12 ? 2 : (N >= 9 ? 5 : 20);
        for (int t = 1; t <= ntiles && e == hipSuccess; ++t) {
            if (!mfma_tile_valid(planes, t, N)) continue;
            double sc = 1.0 / (double)(1u << N);
            e = launch_mfma(FORWARD, planes, in, false, out, false, N, 1, sc, t, ws, s);  // warm-up
            if (e != hipSuccess) break;
            e = hipEventRecord(a, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = launch_mfma(FORWARD, planes, in, false, out, false, N, 1, sc, t, ws, s);
            if (e == hipSuccess) e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e != hipSuccess) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        (void)hipFree(in);
        (void)hipFree(out);
        (void)hipFree(ws);
        if (e != hipSuccess) return hip_fail(e, fn);
        if (best > 0) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            load_tune_cache_locked();
            g_tune[{o.algo, N}] = best;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!save_tune_cache_locked())
            return fail(PAULI_EINVAL, "%s: cannot write %s", fn, getenv("PAULI_TUNE_CACHE"));
    }
    g_last_error.clear();
    return PAULI_OK;
}

// ---------------------------------------------------------------------------
// Coefficients of a list of Pauli strings.  Host plan: sort the strings by
// line group (x >> 4) and low mask bits, cut each group into chunks of at most
// STRINGS_PER_CHUNK, copy [chunks | entries] into the workspace from pinned
// staging, launch one workgroup per chunk.
// ---------------------------------------------------------------------------
namespace {

struct StringsPlan {
    std::vector<StringChunk> chunks;
    std::vector<StringEntry> entries;
    std::vector<uint32_t> first;   // 2^N + 1 offsets: the strings of flip mask x are entries[first[x] .. first[x+1])
    int parts = 1;   // workgroups per chunk (column split), see strings_parts
};

// Split the columns of each chunk over several workgroups when there are too
// few chunks to fill the device: about STRINGS_MAX_BLOCKS workgroups in all.
int strings_parts(int N, size_t nchunks) {
    const size_t want = (size_t)STRINGS_MAX_BLOCKS / nchunks;
    const size_t cap = strings_batches(N);
    const size_t p = want < cap ? want : cap;
    return p < 1 ? 1 : (int)p;
}

size_t strings_ws_bytes(size_t nchunks, size_t count, int parts) {
    return round256(sizeof(StringChunk) * nchunks) + round256(sizeof(StringEntry) * count) +
           (parts > 1 ? round256(sizeof(double) * 2 * count * (size_t)parts) : 0);
}

// Counting sort of the list by flip mask (stable, O(count + 2^N)), then cut
// every line group into chunks.
StringsPlan plan_strings(int N, const uint32_t* strings, int count) {
    StringsPlan P;
    const uint32_t nx = 1u << N;
    std::vector<uint32_t> start(nx + 1, 0u), xs(count);
    for (int k = 0; k < count; ++k) {
        xs[k] = flip_of_index(strings[k]);
        ++start[xs[k] + 1];
    }
    for (uint32_t x = 0; x < nx; ++x) start[x + 1] += start[x];
    std::vector<uint32_t> order(count);
    {
        std::vector<uint32_t> fill(start.begin(), start.end() - 1);
        for (int k = 0; k < count; ++k) order[fill[xs[k]]++] = (uint32_t)k;
    }
    P.entries.resize(count);
    for (int a = 0; a < count; ++a) P.entries[a] = {strings[order[a]], order[a]};
    P.first = start;
    const uint32_t W = N < 4 ? nx : 16u;           // masks per line group
    for (uint32_t g0 = 0; g0 < nx; g0 += W) {
        const uint32_t a0 = start[g0], a1 = start[g0 + W];
        for (uint32_t a = a0; a < a1; a += STRINGS_PER_CHUNK) {
            const uint32_t b = std::min(a1, a + (uint32_t)STRINGS_PER_CHUNK);
            P.chunks.push_back({g0, a, b - a, 0u});
        }
    }
    P.parts = strings_parts(N, P.chunks.size());
    return P;
}

// Pinned host staging for the plan, reused across calls once the copy that
// last read it has completed.
std::mutex g_stage_mu;
void* g_stage = nullptr;
size_t g_stage_bytes = 0;
hipEvent_t g_stage_done = nullptr;

}  // namespace

// Copy host bytes [a | b] (b at offset off_b) into device memory at dst on
// stream s through the shared pinned staging buffer.
static hipError_t stage_copy(void* dst, const void* a, size_t na, const void* b, size_t nb, size_t off_b, hipStream_t s) {
    const size_t bytes = off_b + nb;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    hipError_t e;
    if (!g_stage_done) {
        if ((e = hipEventCreateWithFlags(&g_stage_done, hipEventDisableTiming)) != hipSuccess) {
            g_stage_done = nullptr;
            return e;
        }
    }
    if ((e = hipEventSynchronize(g_stage_done)) != hipSuccess) return e;
    if (g_stage_bytes < bytes) {
        if (g_stage) (void)hipHostFree(g_stage);
        g_stage = nullptr;
        g_stage_bytes = 0;
        if ((e = hipHostMalloc(&g_stage, bytes)) != hipSuccess) {
            g_stage = nullptr;
            return e;
        }
        g_stage_bytes = bytes;
    }
    memcpy(g_stage, a, na);
    memcpy((char*)g_stage + off_b, b, nb);
    if ((e = hipMemcpyAsync(dst, g_stage, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    return hipEventRecord(g_stage_done, s);
}

extern "C" size_t pauli_coeffs_at_workspace_bytes(int N, int count) {
    if (count < 1 || N < 0 || N > N_MAX) return 0;
    const size_t adjoint = round256(sizeof(StringEntry) * (size_t)count) + round256(sizeof(uint32_t) * (((size_t)1 << N) + 1));
    // chunks <= count; the column split gives chunks x parts <= STRINGS_MAX_BLOCKS
    // with chunks >= count / STRINGS_PER_CHUNK, so parts x count stays below
    // STRINGS_MAX_BLOCKS x STRINGS_PER_CHUNK + count, and parts <= strings_batches(N).
    const size_t c = (size_t)count;
    size_t pc = std::min(c * strings_batches(N), (size_t)STRINGS_MAX_BLOCKS * STRINGS_PER_CHUNK + c);
    const size_t forward =
        round256(sizeof(StringChunk) * c) + round256(sizeof(StringEntry) * c) + round256(sizeof(double) * 2 * pc);
    return std::max(forward, adjoint);
}

extern "C" int pauli_coeffs_at(const void* G, int N, const unsigned int* strings, int count, void* out,
                               const pauli_opts* opts) {
    const char* fn = "pauli_coeffs_at";
    const pauli_opts o = resolve(opts);
    if (N < 0 || N > N_MAX) return fail(PAULI_EINVAL, "%s: N=%d outside [0, %d]", fn, N, N_MAX);
    if (count < 1) return fail(PAULI_EINVAL, "%s: count=%d must be >= 1", fn, count);
    if (!G || !out || !strings) return fail(PAULI_EINVAL, "%s: NULL pointer", fn);
    if (!valid_dtype(o.in_dtype) || !valid_dtype(o.out_dtype))
        return fail(PAULI_EINVAL, "%s: unknown dtype (in %d, out %d)", fn, o.in_dtype, o.out_dtype);
    if ((uintptr_t)G % 16 || (uintptr_t)out % 16) return fail(PAULI_EINVAL, "%s: G or out not 16-byte aligned", fn);
    const uint64_t nmax = (uint64_t)1 << (2 * N);
    for (int k = 0; k < count; ++k)
        if ((uint64_t)strings[k] >= nmax)
            return fail(PAULI_EINVAL, "%s: strings[%d]=%u is not below 4^%d", fn, k, strings[k], N);
    const size_t gbytes = (size_t)nmax * elem_bytes(o.in_dtype), obytes = (size_t)count * elem_bytes(o.out_dtype);
    if (overlaps(G, gbytes, out, obytes)) return fail(PAULI_EINVAL, "%s: input and output overlap", fn);
    const StringsPlan P = plan_strings(N, strings, count);
    const size_t need = strings_ws_bytes(P.chunks.size(), P.entries.size(), P.parts);
    if (o.workspace) {
        if ((uintptr_t)o.workspace % 256) return fail(PAULI_EINVAL, "%s: workspace must be 256-byte aligned", fn);
        if (o.workspace_bytes < need)
            return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, o.workspace_bytes);
        if (overlaps(o.workspace, need, G, gbytes) || overlaps(o.workspace, need, out, obytes))
            return fail(PAULI_EINVAL, "%s: workspace overlaps input or output", fn);
    }
    hipStream_t s = (hipStream_t)o.stream;
    hipError_t e;
    void* ws = o.workspace;
    hipMemPool_t pool = nullptr;
    if (!ws) {
        if ((e = pool_for_current_device(&pool)) != hipSuccess) return hip_fail(e, fn);
        if ((e = hipMallocFromPoolAsync(&ws, need, pool, s)) != hipSuccess) return hip_fail(e, fn);
    }
    const size_t chunk_bytes = round256(sizeof(StringChunk) * P.chunks.size());
    const size_t plan_bytes = chunk_bytes + round256(sizeof(StringEntry) * P.entries.size());
    if ((e = stage_copy(ws, P.chunks.data(), sizeof(StringChunk) * P.chunks.size(), P.entries.data(),
                        sizeof(StringEntry) * P.entries.size(), chunk_bytes, s)) != hipSuccess)
        goto fail_free;
    e = launch_strings(G, o.in_dtype == PAULI_C128, N, (const StringChunk*)ws, (int)P.chunks.size(),
                       (const StringEntry*)((char*)ws + chunk_bytes), count, P.parts,
                       (double2*)((char*)ws + plan_bytes), out, o.out_dtype == PAULI_C128, s);
fail_free:
    if (pool) {
        const hipError_t ef = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = ef;
    }
    if (e != hipSuccess) return hip_fail(e, fn);
    g_last_error.clear();
    return PAULI_OK;
}

extern "C" int pauli_coeffs_at_backward(const void* grad_c, int N, const unsigned int* strings, int count,
                                        void* grad_G, const pauli_opts* opts) {
    const char* fn = "pauli_coeffs_at_backward";
    const pauli_opts o = resolve(opts);
    if (N < 0 || N > N_MAX) return fail(PAULI_EINVAL, "%s: N=%d outside [0, %d]", fn, N, N_MAX);
    if (count < 1) return fail(PAULI_EINVAL, "%s: count=%d must be >= 1", fn, count);
    if (!grad_c || !grad_G || !strings) return fail(PAULI_EINVAL, "%s: NULL pointer", fn);
    if (!valid_dtype(o.in_dtype) || !valid_dtype(o.out_dtype))
        return fail(PAULI_EINVAL, "%s: unknown dtype (in %d, out %d)", fn, o.in_dtype, o.out_dtype);
    if ((uintptr_t)grad_c % 16 || (uintptr_t)grad_G % 16)
        return fail(PAULI_EINVAL, "%s: grad_c or grad_G not 16-byte aligned", fn);
    const uint64_t nmax = (uint64_t)1 << (2 * N);
    for (int k = 0; k < count; ++k)
        if ((uint64_t)strings[k] >= nmax)
            return fail(PAULI_EINVAL, "%s: strings[%d]=%u is not below 4^%d", fn, k, strings[k], N);
    const size_t cbytes = (size_t)count * elem_bytes(o.in_dtype), gbytes = (size_t)nmax * elem_bytes(o.out_dtype);
    if (overlaps(grad_c, cbytes, grad_G, gbytes)) return fail(PAULI_EINVAL, "%s: input and output overlap", fn);
    const StringsPlan P = plan_strings(N, strings, count);
    const size_t ent_bytes = round256(sizeof(StringEntry) * P.entries.size());
    const size_t need = ent_bytes + round256(sizeof(uint32_t) * P.first.size());
    if (o.workspace) {
        if ((uintptr_t)o.workspace % 256) return fail(PAULI_EINVAL, "%s: workspace must be 256-byte aligned", fn);
        if (o.workspace_bytes < need)
            return fail(PAULI_ENOMEM, "%s: workspace of %zu bytes needed, %zu given", fn, need, o.workspace_bytes);
        if (overlaps(o.workspace, need, grad_c, cbytes) || overlaps(o.workspace, need, grad_G, gbytes))
            return fail(PAULI_EINVAL, "%s: workspace overlaps input or output", fn);
    }
    hipStream_t s = (hipStream_t)o.stream;
    hipError_t e;
    void* ws = o.workspace;
    hipMemPool_t pool = nullptr;
    if (!ws) {
        if ((e = pool_for_current_device(&pool)) != hipSuccess) return hip_fail(e, fn);
        if ((e = hipMallocFromPoolAsync(&ws, need, pool, s)) != hipSuccess) return hip_fail(e, fn);
    }
    e = stage_copy(ws, P.entries.data(), sizeof(StringEntry) * P.entries.size(), P.first.data(),
                   sizeof(uint32_t) * P.first.size(), ent_bytes, s);
    if (e == hipSuccess)
        e = launch_strings_adjoint(grad_c, o.in_dtype == PAULI_C128, (const StringEntry*)ws,
                                   (const uint32_t*)((char*)ws + ent_bytes), grad_G, o.out_dtype == PAULI_C128, N, s);
    if (pool) {
        const hipError_t ef = hipFreeAsync(ws, s);
        if (e == hipSuccess) e = ef;
    }
    if (e != hipSuccess) return hip_fail(e, fn);
    g_last_error.clear();
    return PAULI_OK;
}
