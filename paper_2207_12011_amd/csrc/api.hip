// api.hip -- host side of the C ABI declared in include/raypc.h.
//
// Owns the per-device context, the resident volumes (brick-ordered level data,
// min/max tables, cached skip bits), brush / transfer-function / option state,
// argument validation and error reporting, and the dispatch of the kernels in
// preprocess.hip and raymarch.hip.  No compute happens on the host apart from
// the camera basis, the level-of-detail choice and small table preparation.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/raypc.h"
#include "context.h"
#include "internal.h"
#include "server.h"

using namespace raypc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? RAYPC_ERR_NOMEM : RAYPC_ERR_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Switches the calling thread to the context's device for the scope.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace {

size_t storage_bytes(int storage) { return storage == kF32 ? 4 : (storage == kF16 ? 2 : 1); }

void free_volume(Volume* v) {
    for (auto& L : v->lv)
        for (auto& users : L.skip_users)
            for (auto& u : users) (void)hipEventDestroy(u.done);
    for (void* p : v->allocs) (void)hipFree(p);
    delete v;
}

int dev_alloc(Volume* v, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(RAYPC_ERR_NOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    v->allocs.push_back(*p);
    v->bytes += bytes;
    return RAYPC_OK;
}

Volume* find_volume(const raypc_ctx* ctx, int id) {
    auto it = ctx->vols.find(id);
    return it == ctx->vols.end() ? nullptr : it->second;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Camera basis in double precision, rounded to float for the kernels.
int camera_setup(const raypc_camera* cam, int width, int height, RenderArgs& a) {
    if (!cam) return fail(RAYPC_ERR_INVALID, "camera is NULL");
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up) || !std::isfinite(cam->fov_y_deg))
        return fail(RAYPC_ERR_INVALID, "camera has a non-finite component");
    if (!(cam->fov_y_deg > 0.0f && cam->fov_y_deg < 180.0f))
        return fail(RAYPC_ERR_INVALID, "fov_y_deg %g outside (0, 180)", cam->fov_y_deg);
    double f[3], u[3], r[3], t[3];
    for (int k = 0; k < 3; ++k) {
        f[k] = static_cast<double>(cam->target[k]) - cam->eye[k];
        u[k] = cam->up[k];
    }
    const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    const double ul = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(fl > 0.0) || !(ul > 0.0)) return fail(RAYPC_ERR_INVALID, "camera eye == target or up is zero");
    for (int k = 0; k < 3; ++k) f[k] /= fl;
    r[0] = f[1] * u[2] - f[2] * u[1];
    r[1] = f[2] * u[0] - f[0] * u[2];
    r[2] = f[0] * u[1] - f[1] * u[0];
    const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 1e-6 * ul)) return fail(RAYPC_ERR_INVALID, "camera up is parallel to the view direction");
    for (int k = 0; k < 3; ++k) r[k] /= rl;
    t[0] = r[1] * f[2] - r[2] * f[1];
    t[1] = r[2] * f[0] - r[0] * f[2];
    t[2] = r[0] * f[1] - r[1] * f[0];
    const double th = std::tan(0.5 * static_cast<double>(cam->fov_y_deg) * M_PI / 180.0);
    double oo = 0.0;
    for (int k = 0; k < 3; ++k) {
        a.eye[k] = cam->eye[k];
        a.fwd[k] = static_cast<float>(f[k]);
        a.right[k] = static_cast<float>(r[k]);
        a.upv[k] = static_cast<float>(t[k]);
        oo += static_cast<double>(cam->eye[k]) * cam->eye[k];
    }
    a.sx_scale = static_cast<float>(th * width / height);
    a.sy_scale = static_cast<float>(th);
    a.inv_w2 = static_cast<float>(2.0 / width);
    a.inv_h2 = static_cast<float>(2.0 / height);
    a.width = width;
    a.height = height;
    a.oo = static_cast<float>(oo);
    return RAYPC_OK;
}

int select_lod_impl(const Volume* v, const raypc_camera* cam, int height, int* lod) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) d2 += static_cast<double>(cam->eye[k]) * cam->eye[k];
    const double dist = std::sqrt(d2);
    const double r = v->r_out;
    if (dist <= r) {
        *lod = 0;
        return RAYPC_OK;
    }
    const double p = height * std::tan(std::asin(r / dist)) / std::tan(0.5 * cam->fov_y_deg * M_PI / 180.0);
    if (!(v->n > p)) {
        *lod = 0;
        return RAYPC_OK;
    }
    const int l = static_cast<int>(std::ceil(std::log2(v->n / p)));
    *lod = std::min(std::max(l, 0), v->n_lods - 1);
    return RAYPC_OK;
}

int check_level(const Volume* v, int lod) {
    if (lod < 0 || lod >= v->n_lods) return fail(RAYPC_ERR_INVALID, "lod %d outside [0, %d]", lod, v->n_lods - 1);
    return RAYPC_OK;
}

}  // namespace

// ============================================================================ internal entry points
namespace raypc {

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

Volume* lookup_volume(raypc_ctx* ctx, int id) { return find_volume(ctx, id); }

void build_skip_args(const raypc_ctx* ctx, const Volume* v, int l, const uint8_t* active, const float* lo,
                     const float* hi, const CoordBrush& coord, int tf_slot, SkipArgs& a) {
    const Level& L = v->lv[l];
    const TFSlot& tf = ctx->tf[tf_slot];
    std::memset(&a, 0, sizeof(a));
    int k = 0;
    for (int f = 0; f < v->nf; ++f) {
        if (!active[f]) continue;
        a.minmax[k] = L.mm[f];
        a.minmax_sub[k] = L.mm_sub[f];
        a.lo[k] = lo[f];
        a.hi[k] = hi[f];
        ++k;
    }
    a.n_active = k;
    a.tf_minmax = L.mm[tf.field];
    a.tf_minmax_sub = L.mm_sub[tf.field];
    a.vmin = tf.vmin;
    a.inv_range = 1.0f / (tf.vmax - tf.vmin);
    int nxt = RAYPC_TF_ENTRIES;
    a.next_nonzero[RAYPC_TF_ENTRIES] = RAYPC_TF_ENTRIES;
    for (int i = RAYPC_TF_ENTRIES - 1; i >= 0; --i) {
        if (tf.rgba[4 * i + 3] > 0.0f) nxt = i;
        a.next_nonzero[i] = nxt;
    }
    a.coord_mask = coord_kernel_form(coord, a.clo, a.chi);
    a.n = L.n;
    a.nb = L.nb;
    a.h = 2.0f / static_cast<float>(L.n);
    a.n_bricks = L.n_bricks();
    a.out_sub = nullptr;
}

// Recompute the skip bits and sub-brick flags of level l for the volume's own brush and a transfer
// slot if stale.
// Record that a launch on `s` read the current skip-flag version of level l (call after the launch).
static int note_use(std::vector<StreamUse>& users, hipStream_t s) {
    StreamUse* u = nullptr;
    for (auto& x : users)
        if (x.stream == s) u = &x;  // later work on a stream completes after its earlier work
    if (!u) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
        users.push_back({s, e});
        u = &users.back();
    }
    HIP_TRY(hipEventRecord(u->done, s), "hipEventRecord(version in use)");
    return RAYPC_OK;
}

// Wait (on the host) until every recorded use of a version has finished, then forget them.
static int wait_uses(std::vector<StreamUse>& users) {
    int rc = RAYPC_OK;
    for (auto& u : users) {
        const hipError_t e = hipEventSynchronize(u.done);
        if (e != hipSuccess && !rc) rc = hip_fail(e, "hipEventSynchronize(version in use)");
    }
    for (auto& u : users) (void)hipEventDestroy(u.done);
    users.clear();
    return rc;
}

static int note_skip_use(Level& L, hipStream_t s) {
    return L.skip_cur < 0 ? RAYPC_OK : note_use(L.skip_users[L.skip_cur], s);
}

// Record that a launch on `s` read the current table version of a transfer-function slot.
static int note_tf_use(raypc_ctx* ctx, int slot, hipStream_t s) {
    TFSlot& t = ctx->tf[slot];
    return t.version < 0 ? RAYPC_OK : note_use(t.users[t.version], s);
}

static int ensure_skip(raypc_ctx* ctx, Volume* v, int l, int slot, hipStream_t s) {
    Level& L = v->lv[l];
    const TFSlot& tf = ctx->tf[slot];
    if (L.skip_valid && L.skip_brush_gen == v->brush_gen && L.skip_slot == slot && L.skip_tf_gen == tf.gen)
        return RAYPC_OK;
    // the next version: wait (on the host) only for the launches that read it when it was current,
    // long ago in the usual case; a render on another stream may still read the current version
    const int next = (L.skip_cur + 1) % kSkipVersions;
    {
        const int rc = wait_uses(L.skip_users[next]);
        if (rc) return rc;
    }
    SkipArgs a;
    build_skip_args(ctx, v, l, v->active, v->lo, v->hi, v->coord, slot, a);
    a.out_sub = L.skip_ver[next];
    HIP_TRY(launch_skip(a, s), "skip-list kernel launch");
    L.skip_cur = next;
    L.skip_sub = L.skip_ver[next];
    L.skip_valid = true;
    L.skip_brush_gen = v->brush_gen;
    L.skip_slot = slot;
    L.skip_tf_gen = tf.gen;
    return RAYPC_OK;
}

uint32_t coord_kernel_form(const CoordBrush& c, float clo[4], float chi[4]) {
    uint32_t mask = 0;
    for (int ax = 0; ax < 4; ++ax) {
        clo[ax] = c.lo[ax];
        chi[ax] = c.hi[ax];
        if (c.active[ax]) mask |= 1u << ax;
    }
    // radius: compared on squares, r^2 >= lo^2 (lo > 0) and r^2 <= hi^2 (hi >= 0; nothing when hi < 0)
    clo[3] = c.lo[3] > 0.0f ? c.lo[3] * c.lo[3] : -INFINITY;
    chi[3] = c.hi[3] >= 0.0f ? c.hi[3] * c.hi[3] : -1.0f;
    return mask;
}

// Greedy test order: after the fields chosen so far, the field that the fewest sampled cells still
// passing them pass, ties to the lower field index.  Only cells whose sub-brick's value range meets
// every brushed interval count (the skip rule drops the samples of the other sub-bricks before any
// fetch).  A sample that fails a brush test fetches no
// further field, so this keeps the expected number of fields fetched per sample low when fields are
// correlated (a field that mostly rejects the same samples as one already tested saves little).
// 8 bytes holding 0 or 1 -> 8 bits (byte j -> bit j).
static inline uint64_t pack8(const uint8_t* b) {
    uint64_t x;
    std::memcpy(&x, b, 8);
    return (x * 0x0102040810204080ull) >> 56;
}

void brush_order(Volume* v, const uint8_t* active, const float* lo, const float* hi, int* order, int& n_brushed) {
    int fields[kMaxFields], m = 0;
    for (int f = 0; f < v->nf; ++f)
        if (active[f]) fields[m++] = f;
    n_brushed = m;
    const int k = v->order_k, words = (k + 63) / 64;
    if (m <= 1 || k == 0) {
        for (int i = 0; i < m; ++i) order[i] = fields[i];
        return;
    }
    if (v->order_cached) {
        bool same = true;
        for (int f = 0; f < v->nf && same; ++f)
            same = v->order_active[f] == (active[f] ? 1 : 0) &&
                   (!active[f] || (v->order_lo[f] == lo[f] && v->order_hi[f] == hi[f]));
        if (same) {
            for (int i = 0; i < m; ++i) order[i] = v->order_fields[i];
            return;
        }
    }
    constexpr int kWords = (kOrderSample + 63) / 64;
    uint64_t pass[kMaxFields][kWords] = {}, alive[kWords], kept[kWords];
    alignas(64) uint8_t pb[kWords * 64] = {}, kb[kWords * 64] = {};
    for (int w = 0; w < words; ++w) kept[w] = ~0ull;
    for (int i = 0; i < m; ++i) {
        const size_t o = static_cast<size_t>(fields[i]) * k;
        const float* x = &v->order_sample[o];
        const float* slo = &v->order_sub_lo[o];
        const float* shi = &v->order_sub_hi[o];
        const float l = lo[fields[i]], h = hi[fields[i]];
        for (int c = 0; c < k; ++c) pb[c] = (x[c] >= l) & (x[c] <= h);
        for (int c = 0; c < k; ++c) kb[c] = (slo[c] <= h) & (shi[c] >= l);
        for (int w = 0; w < words; ++w) {
            uint64_t p = 0, q = 0;
            for (int j = 0; j < 8; ++j) {
                p |= pack8(pb + w * 64 + 8 * j) << (8 * j);
                q |= pack8(kb + w * 64 + 8 * j) << (8 * j);
            }
            pass[i][w] = p;
            kept[w] &= l <= h ? q : 0;  // an empty interval keeps nothing
        }
    }
    for (int w = 0; w < words; ++w) alive[w] = kept[w];
    bool used[kMaxFields] = {};
    for (int pos = 0; pos < m; ++pos) {
        int best = -1, best_count = 0;
        for (int i = 0; i < m; ++i) {
            if (used[i]) continue;
            int cnt = 0;
            for (int w = 0; w < words; ++w) cnt += __builtin_popcountll(alive[w] & pass[i][w]);
            if (best < 0 || cnt < best_count) {
                best = i;
                best_count = cnt;
            }
        }
        used[best] = true;
        order[pos] = fields[best];
        for (int w = 0; w < words; ++w) alive[w] &= pass[best][w];
    }
    v->order_cached = true;
    for (int f = 0; f < v->nf; ++f) {
        v->order_active[f] = active[f] ? 1 : 0;
        v->order_lo[f] = lo[f];
        v->order_hi[f] = hi[f];
    }
    for (int i = 0; i < m; ++i) v->order_fields[i] = order[i];
    v->order_n = m;
}

int prepare_render(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                   float step, const uint8_t* brush_active, const float* brush_lo, const float* brush_hi,
                   const CoordBrush& coord, int tf_slot, float* rgba_out, bool use_volume_state, hipStream_t s,
                   RenderArgs& a, int& storage, int& level, Volume** vol_out) {
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    if (width < 1 || width > 16384 || height < 1 || height > 16384)
        return fail(RAYPC_ERR_INVALID, "image size %dx%d outside [1, 16384]", width, height);
    if (!(step >= 1.0f / 64.0f && step <= 64.0f)) return fail(RAYPC_ERR_INVALID, "step %g outside [1/64, 64]", step);
    if (!rgba_out) return fail(RAYPC_ERR_INVALID, "rgba_out is NULL");
    if (reinterpret_cast<uintptr_t>(rgba_out) % 16 != 0) return fail(RAYPC_ERR_INVALID, "rgba_out must be 16-byte aligned");
    if (tf_slot < 0 || tf_slot >= RAYPC_TF_SLOTS || !ctx->tf[tf_slot].defined)
        return fail(RAYPC_ERR_INVALID, "transfer-function slot %d is not defined", tf_slot);
    const TFSlot& tf = ctx->tf[tf_slot];
    if (tf.field >= v->nf)
        return fail(RAYPC_ERR_INVALID, "transfer function classifies field %d but the volume has %d", tf.field, v->nf);
    for (int f = 0; f < v->nf; ++f)
        if (brush_active[f] && (std::isnan(brush_lo[f]) || std::isnan(brush_hi[f])))
            return fail(RAYPC_ERR_INVALID, "NaN bound for field %d", f);
    for (int ax = 0; ax < 4; ++ax)
        if (coord.active[ax] && (std::isnan(coord.lo[ax]) || std::isnan(coord.hi[ax])))
            return fail(RAYPC_ERR_INVALID, "NaN bound for coordinate axis %d", ax);
    std::memset(&a, 0, sizeof(a));
    a.coord_mask = coord_kernel_form(coord, a.clo, a.chi);
    int rc = camera_setup(cam, width, height, a);
    if (rc) return rc;
    if (lod == -1) select_lod_impl(v, cam, height, &lod);
    rc = check_level(v, lod);
    if (rc) return rc;
    const Level& L = v->lv[lod];

    int order[kMaxFields], n_brushed = 0;
    brush_order(v, brush_active, brush_lo, brush_hi, order, n_brushed);
    int k = 0;
    bool tf_brushed = false;
    for (int i = 0; i < n_brushed; ++i) {
        const int f = order[i];
        a.field[k] = L.data[f];
        a.u8par[k] = L.par[f];
        a.rec[k] = L.rec[f];
        // binary16 codes hold the field times 2^k: the march compares them with the bounds times 2^k,
        // which decides exactly as the values against the bounds (powers of two scale exactly)
        a.lo[k] = brush_lo[f] * stored_scale(v, f);
        a.hi[k] = brush_hi[f] * stored_scale(v, f);
        if (f == tf.field) {
            a.tf_slot = k;
            tf_brushed = true;
        }
        ++k;
    }
    a.n_brushed = k;
    if (!tf_brushed) {
        a.tf_slot = k;
        a.field[k] = L.data[tf.field];
        a.u8par[k] = L.par[tf.field];
        a.rec[k] = L.rec[tf.field];
    }
    a.n = L.n;
    a.nb = L.nb;
    {
        const uint64_t fb = v->storage == kU8    ? u8_field_bytes(L.nb)
                            : v->storage == kF16 ? f16_field_bytes(L.nb)
                                                 : static_cast<uint64_t>(L.n) * L.n * L.n * storage_bytes(v->storage);
        a.field_bytes = fb > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(fb);
        a.par_bytes = static_cast<uint32_t>((L.n_bricks() + 1) * sizeof(float2));   // with the zero pair after the last brick
        const uint64_t rb = record_bytes(L.nb);
        a.rec_bytes = rb > 0xFFFFFFFFull ? 0xFFFFFFFFu : static_cast<uint32_t>(rb);
    }
    a.half_n = 0.5f * static_cast<float>(L.n);
    a.tf = tf.dev;
    // the table's index map of the scaled values: (s v - s vmin) (inv / s) = (v - vmin) inv exactly
    a.vmin = tf.vmin * stored_scale(v, tf.field);
    a.inv_range = (1.0f / (tf.vmax - tf.vmin)) / stored_scale(v, tf.field);
    a.inv_ref = 1.0f / tf.ref_step;
    a.ert = ctx->ert;
    a.ert_on = ctx->ert < 1.0f;
    for (int c = 0; c < 4; ++c) a.bg[c] = ctx->bg[c];
    a.has_bg = ctx->has_bg;
    a.r_in2 = v->r_in * v->r_in;
    a.r_out2 = v->r_out * v->r_out;
    a.c_in = a.oo - a.r_in2;
    a.c_out = a.oo - a.r_out2;
    a.has_inner = v->r_in > 0.0f;
    a.ds = step * (2.0f / static_cast<float>(L.n));
    a.inv_ds = 1.0f / a.ds;
    a.out = reinterpret_cast<float4*>(rgba_out);
    // single-image launches take the context's wave tile shape; serving steps keep 4 x 4 tiles
    a.tile_log2w = use_volume_state ? ctx->tile_log2w : kDefaultTileLog2W;
    {
        const int tw = 1 << a.tile_log2w, th = 16 >> a.tile_log2w;
        a.blocks_x = (width + tw - 1) / tw;
        a.n_blocks = a.blocks_x * ((height + th - 1) / th);
    }
    a.super_log2 = ctx->super_log2;
    a.skip = nullptr;
    if (use_volume_state) {
        rc = ensure_skip(ctx, v, lod, tf_slot, s);
        if (rc) return rc;
        a.skip = v->lv[lod].skip_sub;
    }
    // kernel kind
    storage = !v->records ? v->storage : (v->storage == kF32 ? kKindF32Rec : v->storage == kF16 ? kKindF16Rec : kKindU8Rec);
    level = lod;
    if (vol_out) *vol_out = v;
    return RAYPC_OK;
}

}  // namespace raypc

// ============================================================================ C ABI
extern "C" {

int raypc_version(void) { return 10000; }

const char* raypc_last_error(void) { return g_last_error.c_str(); }

int raypc_create(int device, raypc_ctx** out) {
    if (!out) return fail(RAYPC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(RAYPC_ERR_INVALID, "device %d outside [0, %d)", device, count);
    DeviceGuard g(device);
    // the allocation-free warp's fixed z-buffer on this device (looked up with the device current)
    unsigned long long* scratch_keys = nullptr;
    e = warp_scratch(device, &scratch_keys);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(warp scratch z-buffer)");
    raypc_ctx* ctx = new raypc_ctx();
    ctx->device = device;
    ctx->warp_scratch = scratch_keys;
    for (int s = 0; s < RAYPC_TF_SLOTS; ++s) {
        e = hipMalloc(reinterpret_cast<void**>(&ctx->tf[s].pool), size_t(kTFVersions) * RAYPC_TF_ENTRIES * sizeof(float4));
        if (e != hipSuccess) {
            for (int t = 0; t < s; ++t) (void)hipFree(ctx->tf[t].pool);
            delete ctx;
            return hip_fail(e, "hipMalloc(transfer-function tables)");
        }
    }
    e = hipStreamCreateWithFlags(&ctx->upload, hipStreamNonBlocking);
    if (e != hipSuccess) {
        for (auto& t : ctx->tf) {
        for (auto& users : t.users)
            for (auto& u : users) (void)hipEventDestroy(u.done);
        (void)hipFree(t.pool);
    }
        delete ctx;
        return hip_fail(e, "hipStreamCreateWithFlags(upload stream)");
    }
    *out = ctx;
    return RAYPC_OK;
}

void raypc_destroy(raypc_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard g(ctx->device);
    server_shutdown(ctx);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->vols) free_volume(kv.second);
    for (auto& t : ctx->tf) {
        for (auto& users : t.users)
            for (auto& u : users) (void)hipEventDestroy(u.done);
        (void)hipFree(t.pool);
    }
    if (ctx->upload) (void)hipStreamDestroy(ctx->upload);
    if (ctx->tf_stage) (void)hipHostFree(ctx->tf_stage);
    for (auto* k : ctx->warp_keys)
        if (k) (void)hipFree(k);
    delete ctx;
}

int raypc_load_fields(raypc_ctx* ctx, int n_fields, int n, const float* const* fields, int on_device, int storage,
                      int n_lods, float r_inner, float r_outer, void* stream, int* volume_id) {
    if (!ctx || !fields || !volume_id) return fail(RAYPC_ERR_INVALID, "NULL argument");
    if (n_fields < 1 || n_fields > RAYPC_MAX_FIELDS) return fail(RAYPC_ERR_INVALID, "n_fields %d outside [1, 8]", n_fields);
    if (n < 32 || n > 1024 || n % 32 != 0) return fail(RAYPC_ERR_INVALID, "n %d must be a multiple of 32 in [32, 1024]", n);
    const int storage_arg = storage;
    const bool compact = (storage & RAYPC_STORAGE_COMPACT) != 0;
    storage &= ~RAYPC_STORAGE_COMPACT;
    if (storage < RAYPC_STORAGE_F32 || storage > RAYPC_STORAGE_U8_BRICK)
        return fail(RAYPC_ERR_INVALID, "storage %d unknown", storage_arg);
    if (n_lods < 1 || n_lods > RAYPC_MAX_LODS) return fail(RAYPC_ERR_INVALID, "n_lods %d outside [1, 3]", n_lods);
    if (!(r_inner >= 0.0f && r_inner < r_outer && r_outer <= 1.0f))
        return fail(RAYPC_ERR_INVALID, "radii must satisfy 0 <= r_inner < r_outer <= 1");
    for (int f = 0; f < n_fields; ++f)
        if (!fields[f]) return fail(RAYPC_ERR_INVALID, "fields[%d] is NULL", f);
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nvox = static_cast<size_t>(n) * n * n;

    Volume* v = new Volume();
    v->n = n;
    v->nf = n_fields;
    v->n_lods = n_lods;
    v->storage = storage;
    v->records = !compact;
    v->r_in = r_inner;
    v->r_out = r_outer;
    for (int f = 0; f < n_fields; ++f) {
        v->lo[f] = -INFINITY;
        v->hi[f] = INFINITY;
    }
    int rc = RAYPC_OK;
    // scratch: host-input staging (one field), two level buffers, a flag
    std::vector<void*> tmp;
    auto tmp_alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(RAYPC_ERR_NOMEM, "scratch allocation of %zu bytes failed", bytes);
        }
        tmp.push_back(*p);
        return RAYPC_OK;
    };
    float* stage = nullptr;
    float* lvbuf[2] = {nullptr, nullptr};
    unsigned int* flag = nullptr;
    unsigned int* maxbits = nullptr;
    float* f16_scales = nullptr;
    int* f16_exps = nullptr;
    // shell cells whose values estimate each brush's field selectivities: uniform over the cells whose
    // centre lies in the shell, drawn with a SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014)
    std::vector<uint32_t> cells;
    {
        uint64_t z = 0x2207120110ull;
        const double h = 2.0 / n;
        for (int tries = 0; static_cast<int>(cells.size()) < kOrderSample && tries < 64 * kOrderSample; ++tries) {
            z += 0x9E3779B97F4A7C15ull;
            uint64_t r = z;
            r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
            r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
            r ^= r >> 31;
            const uint32_t i = static_cast<uint32_t>(r % nvox);
            const double x = (i % n + 0.5) * h - 1.0, y = ((i / n) % n + 0.5) * h - 1.0;
            const double zc = (i / (static_cast<size_t>(n) * n) + 0.5) * h - 1.0;
            const double rad = std::sqrt(x * x + y * y + zc * zc);
            if (rad >= r_inner && rad <= r_outer) cells.push_back(i);
        }
    }
    const int n_cells = static_cast<int>(cells.size());
    std::vector<uint32_t> cell_sub(cells.size());  // index of each cell's sub-brick in the level-0 tables
    for (int c = 0; c < n_cells; ++c) {
        const uint32_t i = cells[c], x = i % n, y = (i / n) % n, zc = i / (static_cast<uint32_t>(n) * n);
        const uint32_t nbk = static_cast<uint32_t>(n / kBrick);
        const uint32_t brick = ((zc >> 3) * nbk + (y >> 3)) * nbk + (x >> 3);
        cell_sub[c] = brick * 8 + (((x >> 2) & 1) | (((y >> 2) & 1) << 1) | (((zc >> 2) & 1) << 2));
    }
    uint32_t* d_cells = nullptr;
    uint32_t* d_cell_sub = nullptr;
    float* d_sample = nullptr;
    float2* d_sub = nullptr;
    do {
        for (int l = 0; l < n_lods && !rc; ++l) {
            Level& L = v->lv[l];
            L.n = n >> l;
            L.nb = L.n / kBrick;
            const size_t lvox = static_cast<size_t>(L.n) * L.n * L.n;
            for (int f = 0; f < n_fields && !rc; ++f) {
                rc = dev_alloc(v, &L.data[f], storage == kU8 ? u8_field_bytes(L.nb)
                                              : (storage == kF16 ? f16_field_bytes(L.nb) : lvox * storage_bytes(storage)));
                // one pair more than the bricks, left zero: the ray march reads each brick's pair together
                // with the next one, the last brick's included
                if (!rc && storage == kU8) rc = dev_alloc(v, reinterpret_cast<void**>(&L.par[f]), (L.n_bricks() + 1) * sizeof(float2));
                if (!rc) rc = dev_alloc(v, reinterpret_cast<void**>(&L.mm[f]), L.n_bricks() * sizeof(float2));
                if (!rc) rc = dev_alloc(v, reinterpret_cast<void**>(&L.mm_sub[f]), L.n_bricks() * 8 * sizeof(float2));
                if (!rc && v->records) rc = dev_alloc(v, &L.rec[f], record_bytes(L.nb));
            }
            for (int k = 0; k < kSkipVersions && !rc; ++k)
                rc = dev_alloc(v, reinterpret_cast<void**>(&L.skip_ver[k]), L.n_bricks() * sizeof(uint16_t));
        }
        if (rc) break;
        if (!on_device && (rc = tmp_alloc(reinterpret_cast<void**>(&stage), nvox * sizeof(float)))) break;
        if (n_lods > 1 && (rc = tmp_alloc(reinterpret_cast<void**>(&lvbuf[0]), nvox / 8 * sizeof(float)))) break;
        if (n_lods > 2 && (rc = tmp_alloc(reinterpret_cast<void**>(&lvbuf[1]), nvox / 64 * sizeof(float)))) break;
        if ((rc = tmp_alloc(reinterpret_cast<void**>(&flag), sizeof(unsigned int)))) break;
        // per field: the largest |value| (bits), binary16's scale pair and exponent
        if ((rc = tmp_alloc(reinterpret_cast<void**>(&maxbits), kMaxFields * sizeof(unsigned int)))) break;
        if ((rc = tmp_alloc(reinterpret_cast<void**>(&f16_scales), 2 * kMaxFields * sizeof(float)))) break;
        if ((rc = tmp_alloc(reinterpret_cast<void**>(&f16_exps), kMaxFields * sizeof(int)))) break;
        if (n_cells > 0) {
            if ((rc = tmp_alloc(reinterpret_cast<void**>(&d_cells), n_cells * sizeof(uint32_t)))) break;
            if ((rc = tmp_alloc(reinterpret_cast<void**>(&d_sample), static_cast<size_t>(n_fields) * n_cells * sizeof(float))))
                break;
            if ((rc = tmp_alloc(reinterpret_cast<void**>(&d_cell_sub), n_cells * sizeof(uint32_t)))) break;
            if ((rc = tmp_alloc(reinterpret_cast<void**>(&d_sub), static_cast<size_t>(n_fields) * n_cells * sizeof(float2))))
                break;
            hipError_t ce = hipMemcpyAsync(d_cells, cells.data(), n_cells * sizeof(uint32_t), hipMemcpyHostToDevice, s);
            if (ce == hipSuccess)
                ce = hipMemcpyAsync(d_cell_sub, cell_sub.data(), n_cells * sizeof(uint32_t), hipMemcpyHostToDevice, s);
            if (ce != hipSuccess) { rc = hip_fail(ce, "hipMemcpyAsync(cells)"); break; }
        }
        hipError_t e = hipMemsetAsync(flag, 0, sizeof(unsigned int), s);
        if (e == hipSuccess) e = hipMemsetAsync(maxbits, 0, kMaxFields * sizeof(unsigned int), s);
        if (e == hipSuccess) e = hipMemsetAsync(f16_exps, 0, kMaxFields * sizeof(int), s);
        if (e != hipSuccess) { rc = hip_fail(e, "hipMemsetAsync"); break; }
        for (int f = 0; f < n_fields && !rc; ++f) {
            const float* src = fields[f];
            if (!on_device) {
                e = hipMemcpyAsync(stage, src, nvox * sizeof(float), hipMemcpyHostToDevice, s);
                if (e != hipSuccess) { rc = hip_fail(e, "hipMemcpyAsync(field)"); break; }
                src = stage;
            }
            if ((e = launch_count_nonfinite(src, nvox, flag, maxbits + f, s)) != hipSuccess) { rc = hip_fail(e, "finite check"); break; }
            const float* f16_scale = storage == kF16 ? f16_scales + 2 * f : nullptr;
            if (f16_scale && (e = launch_f16_scale(maxbits + f, f16_scales + 2 * f, f16_exps + f, s)) != hipSuccess) {
                rc = hip_fail(e, "binary16 scale");
                break;
            }
            if ((e = launch_gather_cells(src, d_cells, n_cells, d_sample + static_cast<size_t>(f) * n_cells, s)) != hipSuccess) {
                rc = hip_fail(e, "cell sample");
                break;
            }
            const float* cur = src;
            for (int l = 0; l < n_lods; ++l) {
                Level& L = v->lv[l];
                if (l > 0) {
                    float* nxt = lvbuf[l - 1];
                    if ((e = launch_lod_build(cur, v->lv[l - 1].n, nxt, s)) != hipSuccess) { rc = hip_fail(e, "level build"); break; }
                    cur = nxt;
                }
                if (storage == kU8 && ((e = hipMemsetAsync(L.par[f] + L.n_bricks(), 0, sizeof(float2), s)) != hipSuccess ||
                                       (e = hipMemsetAsync(static_cast<uint8_t*>(L.data[f]) + u8_field_bytes(L.nb) - 16, 0, 16, s)) != hipSuccess)) {
                    rc = hip_fail(e, "8-bit padding");
                    break;
                }
                if (storage == kF16 &&
                    (e = hipMemsetAsync(static_cast<uint8_t*>(L.data[f]) + f16_field_bytes(L.nb) - 16, 0, 16, s)) != hipSuccess) {
                    rc = hip_fail(e, "binary16 padding");
                    break;
                }
                if ((e = launch_encode(cur, L.n, storage, L.data[f], L.par[f], f16_scale, s)) != hipSuccess) { rc = hip_fail(e, "encode"); break; }
                if ((e = launch_minmax(L.data[f], L.par[f], L.n, storage, L.mm[f], L.mm_sub[f], f16_scale, s)) != hipSuccess) { rc = hip_fail(e, "min/max"); break; }
                if (l == 0 && (e = launch_gather_pairs(L.mm_sub[f], d_cell_sub, n_cells, d_sub + static_cast<size_t>(f) * n_cells,
                                                       s)) != hipSuccess) {
                    rc = hip_fail(e, "sub-brick sample");
                    break;
                }
                if (v->records && (e = launch_records(L.data[f], L.par[f], L.n, storage, L.rec[f], s)) != hipSuccess) { rc = hip_fail(e, "neighbourhood records"); break; }
            }
        }
        if (rc) break;
        unsigned int h_flag = 0;
        v->order_sample.resize(static_cast<size_t>(n_fields) * n_cells);
        std::vector<float2> sub_pairs(static_cast<size_t>(n_fields) * n_cells);
        v->order_k = n_cells;
        e = hipMemcpyAsync(&h_flag, flag, sizeof(h_flag), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(v->f16_exp, f16_exps, kMaxFields * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && n_cells > 0)
            e = hipMemcpyAsync(v->order_sample.data(), d_sample, v->order_sample.size() * sizeof(float),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && n_cells > 0)
            e = hipMemcpyAsync(sub_pairs.data(), d_sub, sub_pairs.size() * sizeof(float2), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        v->order_sub_lo.resize(sub_pairs.size());
        v->order_sub_hi.resize(sub_pairs.size());
        for (size_t i = 0; i < sub_pairs.size(); ++i) {
            v->order_sub_lo[i] = sub_pairs[i].x;
            v->order_sub_hi[i] = sub_pairs[i].y;
        }
        if (e != hipSuccess) { rc = hip_fail(e, "load synchronisation"); break; }
        if (h_flag) rc = fail(RAYPC_ERR_INVALID, "input contains a non-finite value");
    } while (0);
    if (!tmp.empty()) (void)hipStreamSynchronize(s);
    for (void* p : tmp) (void)hipFree(p);
    if (rc) {
        free_volume(v);
        return rc;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    v->id = ctx->next_id++;
    ctx->vols[v->id] = v;
    *volume_id = v->id;
    return RAYPC_OK;
}

int raypc_unload(raypc_ctx* ctx, int volume_id) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    if (v->refs > 0) return fail(RAYPC_ERR_BUSY, "volume %d has %d serving requests in flight", volume_id, v->refs);
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->vols.erase(volume_id);
    free_volume(v);
    return RAYPC_OK;
}

int raypc_volume_info(const raypc_ctx* ctx, int volume_id, int* n_fields, int* n, int* n_lods, int* storage,
                      uint64_t* bytes) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    const Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    if (n_fields) *n_fields = v->nf;
    if (n) *n = v->n;
    if (n_lods) *n_lods = v->n_lods;
    if (storage) *storage = v->storage | (v->records ? 0 : RAYPC_STORAGE_COMPACT);
    if (bytes) *bytes = v->bytes;
    return RAYPC_OK;
}

int raypc_set_brush(raypc_ctx* ctx, int volume_id, int n_fields, const uint8_t* active, const float* lo,
                    const float* hi) {
    if (!ctx || !active || !lo || !hi) return fail(RAYPC_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    if (n_fields != v->nf) return fail(RAYPC_ERR_INVALID, "brush has %d fields, volume has %d", n_fields, v->nf);
    for (int f = 0; f < n_fields; ++f)
        if (std::isnan(lo[f]) || std::isnan(hi[f])) return fail(RAYPC_ERR_INVALID, "NaN bound for field %d", f);
    for (int f = 0; f < n_fields; ++f) {
        v->active[f] = active[f] ? 1 : 0;
        v->lo[f] = lo[f];
        v->hi[f] = hi[f];
    }
    ++v->brush_gen;
    return RAYPC_OK;
}

int raypc_set_coordinate_brush(raypc_ctx* ctx, int volume_id, const uint8_t* active, const float* lo, const float* hi) {
    if (!ctx || !active || !lo || !hi) return fail(RAYPC_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    for (int ax = 0; ax < 4; ++ax)
        if (std::isnan(lo[ax]) || std::isnan(hi[ax])) return fail(RAYPC_ERR_INVALID, "NaN bound for axis %d", ax);
    for (int ax = 0; ax < 4; ++ax) {
        v->coord.active[ax] = active[ax] ? 1 : 0;
        v->coord.lo[ax] = lo[ax];
        v->coord.hi[ax] = hi[ax];
    }
    ++v->brush_gen;
    return RAYPC_OK;
}

// Both entry points: `async` enqueues the upload on `stream` (from a pinned staging copy) and returns;
// otherwise the upload runs on the context's own stream and is waited for.
static int set_tf_impl(raypc_ctx* ctx, int slot, int field, float vmin, float vmax, const float* rgba, int n_entries,
                       float ref_step, bool async, hipStream_t stream) {
    if (!ctx || !rgba) return fail(RAYPC_ERR_INVALID, "NULL argument");
    if (slot < 0 || slot >= RAYPC_TF_SLOTS) return fail(RAYPC_ERR_INVALID, "slot %d outside [0, 8)", slot);
    if (n_entries != RAYPC_TF_ENTRIES) return fail(RAYPC_ERR_INVALID, "n_entries must be 256");
    if (field < 0 || field >= RAYPC_MAX_FIELDS) return fail(RAYPC_ERR_INVALID, "field %d outside [0, 8)", field);
    if (!std::isfinite(vmin) || !std::isfinite(vmax) || !(vmax > vmin))
        return fail(RAYPC_ERR_INVALID, "need finite vmin < vmax");
    if (!std::isfinite(1.0f / (vmax - vmin))) return fail(RAYPC_ERR_INVALID, "value range too narrow");
    if (!(ref_step > 0.0f) || !std::isfinite(ref_step)) return fail(RAYPC_ERR_INVALID, "ref_step must be > 0");
    for (int i = 0; i < RAYPC_TF_ENTRIES * 4; ++i)
        if (!(rgba[i] >= 0.0f && rgba[i] <= 1.0f)) return fail(RAYPC_ERR_INVALID, "table entry %d outside [0, 1]", i / 4);
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    TFSlot& t = ctx->tf[slot];
    // the new table goes to the slot's next version: renders already enqueued (on any stream) keep
    // reading the version they were given; renders enqueued after this call read the new one
    const int next = (t.version + 1) % kTFVersions;
    // the launches that read this version, kTFVersions definitions ago, and its upload have finished
    // long since in the usual case; wait for them otherwise
    {
        const int rc = wait_uses(t.users[next]);
        if (rc) return rc;
    }
    float4* dst = t.pool + size_t(next) * RAYPC_TF_ENTRIES;
    hipError_t e = hipSuccess;
    if (async) {
        // a pinned staging copy per (slot, version), reused only after this version's upload (a
        // recorded use) has finished
        if (!ctx->tf_stage) {
            e = hipHostMalloc(reinterpret_cast<void**>(&ctx->tf_stage),
                              size_t(RAYPC_TF_SLOTS) * kTFVersions * RAYPC_TF_ENTRIES * sizeof(float4), hipHostMallocDefault);
            if (e != hipSuccess) {
                ctx->tf_stage = nullptr;
                return hip_fail(e, "hipHostMalloc(transfer-function staging)");
            }
        }
        float4* stage = ctx->tf_stage + (size_t(slot) * kTFVersions + next) * RAYPC_TF_ENTRIES;
        std::memcpy(stage, rgba, RAYPC_TF_ENTRIES * sizeof(float4));
        e = hipMemcpyAsync(dst, stage, RAYPC_TF_ENTRIES * sizeof(float4), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) {
            const int rc = note_use(t.users[next], stream);
            if (rc) return rc;
        }
    } else {
        // on the context's own non-blocking stream: waits for this copy (and for whatever the runtime
        // queued ahead of it on the hardware queue that stream shares), not for a device drain
        e = hipMemcpyAsync(dst, rgba, RAYPC_TF_ENTRIES * sizeof(float4), hipMemcpyHostToDevice, ctx->upload);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->upload);
    }
    if (e != hipSuccess) return hip_fail(e, "transfer-function upload");
    t.version = next;
    t.dev = dst;
    t.defined = true;
    t.field = field;
    t.vmin = vmin;
    t.vmax = vmax;
    t.ref_step = ref_step;
    std::memcpy(t.rgba, rgba, sizeof(t.rgba));
    t.gen = ++ctx->tf_gen_counter;
    return RAYPC_OK;
}

int raypc_set_transfer_function(raypc_ctx* ctx, int slot, int field, float vmin, float vmax, const float* rgba,
                                int n_entries, float ref_step) {
    return set_tf_impl(ctx, slot, field, vmin, vmax, rgba, n_entries, ref_step, false, nullptr);
}

int raypc_set_transfer_function_async(raypc_ctx* ctx, int slot, int field, float vmin, float vmax, const float* rgba,
                                      int n_entries, float ref_step, void* stream) {
    return set_tf_impl(ctx, slot, field, vmin, vmax, rgba, n_entries, ref_step, true, static_cast<hipStream_t>(stream));
}

int raypc_set_options(raypc_ctx* ctx, float ert_threshold, const float* bg_rgba) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    if (!(ert_threshold > 0.0f)) return fail(RAYPC_ERR_INVALID, "ert_threshold must be > 0");
    if (bg_rgba)
        for (int c = 0; c < 4; ++c)
            if (!(bg_rgba[c] >= 0.0f && bg_rgba[c] <= 1.0f)) return fail(RAYPC_ERR_INVALID, "background outside [0, 1]");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->ert = ert_threshold;
    ctx->has_bg = bg_rgba != nullptr;
    for (int c = 0; c < 4; ++c) ctx->bg[c] = bg_rgba ? bg_rgba[c] : 0.0f;
    return RAYPC_OK;
}

int raypc_select_lod(const raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int* lod) {
    if (!ctx || !cam || !lod) return fail(RAYPC_ERR_INVALID, "NULL argument");
    const Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    RenderArgs a;
    int rc = camera_setup(cam, std::max(width, 1), std::max(height, 1), a);
    if (rc) return rc;
    if (width < 1 || height < 1) return fail(RAYPC_ERR_INVALID, "image size must be positive");
    return select_lod_impl(v, cam, height, lod);
}

static int render_common(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                         float step, float* rgba_out, uint32_t* nominal, uint32_t* composited, uint32_t* touched,
                         bool counts, bool use_skip, void* stream, uint32_t* evaluated = nullptr,
                         uint32_t* fetched = nullptr) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    RenderArgs a;
    int storage = 0, level = 0;
    int rc = prepare_render(ctx, volume_id, cam, width, height, lod, step, v->active, v->lo, v->hi, v->coord, 0, rgba_out,
                            true, s, a, storage, level, nullptr);
    if (rc) return rc;
    if (!use_skip) a.skip = nullptr;
    a.nominal = nominal;
    a.composited = composited;
    a.touched = touched;
    a.evaluated = evaluated;
    a.fetched = fetched;
    HIP_TRY(launch_render(a, storage, counts, s), "ray-march kernel launch");
    rc = note_tf_use(ctx, 0, s);
    if (rc) return rc;
    return a.skip ? note_skip_use(v->lv[level], s) : RAYPC_OK;
}

int raypc_render(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod, float step,
                 float* rgba_out, void* stream) {
    return render_common(ctx, volume_id, cam, width, height, lod, step, rgba_out, nullptr, nullptr, nullptr, false, true,
                         stream);
}

int raypc_render_debug(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                       float step, float* rgba_out, uint32_t* nominal, uint32_t* composited, uint32_t* touched_bricks,
                       int flags, void* stream) {
    return render_common(ctx, volume_id, cam, width, height, lod, step, rgba_out, nominal, composited, touched_bricks,
                         true, (flags & 1) == 0, stream);
}

int raypc_render_work(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                      float step, float* rgba_out, uint32_t* evaluated, uint32_t* fetched, void* stream) {
    return render_common(ctx, volume_id, cam, width, height, lod, step, rgba_out, nullptr, nullptr, nullptr, true,
                         true, stream, evaluated, fetched);
}

int raypc_render_jittered(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                          float step, int pass, int n_passes, uint64_t seed, float* rgba_out, float* mean_inout,
                          uint32_t* nominal, uint32_t* composited, void* stream) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    if (n_passes < 1 || n_passes > 256 || pass < 0 || pass >= n_passes)
        return fail(RAYPC_ERR_INVALID, "need 0 <= pass (%d) < n_passes (%d) <= 256", pass, n_passes);
    if (!rgba_out && !mean_inout) return fail(RAYPC_ERR_INVALID, "rgba_out and mean_inout are both NULL");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    RenderArgs a;
    int storage = 0, level = 0;
    // prepare_render checks rgba_out for NULL; the jittered pass may write only the running mean
    float* out = rgba_out ? rgba_out : mean_inout;
    int rc = prepare_render(ctx, volume_id, cam, width, height, lod, step, v->active, v->lo, v->hi, v->coord, 0, out, true, s, a,
                            storage, level, nullptr);
    if (rc) return rc;
    a.out = reinterpret_cast<float4*>(rgba_out);
    a.nominal = nominal;
    a.composited = composited;
    a.touched = nullptr;
    a.seed = seed;
    a.pass = static_cast<uint32_t>(pass);
    a.n_passes = static_cast<uint32_t>(n_passes);
    a.inv_pass1 = 1.0f / static_cast<float>(pass + 1);
    a.mean = reinterpret_cast<float4*>(mean_inout);
    HIP_TRY(launch_render_jittered(a, storage, nominal != nullptr || composited != nullptr, s),
            "jittered ray-march kernel launch");
    rc = note_tf_use(ctx, 0, s);
    if (rc) return rc;
    return note_skip_use(v->lv[level], s);
}

int raypc_render_depth(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                       float step, float* rgba_out, float* depth_out, void* stream) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    if (!depth_out) return fail(RAYPC_ERR_INVALID, "depth_out is NULL");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    RenderArgs a;
    int storage = 0, level = 0;
    int rc = prepare_render(ctx, volume_id, cam, width, height, lod, step, v->active, v->lo, v->hi, v->coord, 0, rgba_out,
                            true, s, a, storage, level, nullptr);
    if (rc) return rc;
    a.depth = depth_out;
    HIP_TRY(launch_render_depth(a, storage, s), "depth ray-march kernel launch");
    rc = note_tf_use(ctx, 0, s);
    if (rc) return rc;
    return note_skip_use(v->lv[level], s);
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return a && b && x < y + nb && y < x + na;
}

// Validation and the camera frames of a warp (both warp entry points); the z-buffers are left to the caller.
static int warp_setup(raypc_ctx* ctx, const raypc_camera* src_cam, int src_width, int src_height, const float* rgba,
                      const float* depth, const raypc_camera* dst_cam, int dst_width, int dst_height, float* rgba_out,
                      float* depth_out, int32_t* source_out, WarpArgs& w) {
    if (!ctx || !rgba || !depth || !rgba_out) return fail(RAYPC_ERR_INVALID, "NULL argument");
    if (src_width < 1 || src_width > 16384 || src_height < 1 || src_height > 16384 || dst_width < 1 ||
        dst_width > 16384 || dst_height < 1 || dst_height > 16384)
        return fail(RAYPC_ERR_INVALID, "image sizes %dx%d -> %dx%d outside [1, 16384]", src_width, src_height,
                    dst_width, dst_height);
    const size_t ns = static_cast<size_t>(src_width) * src_height, nd = static_cast<size_t>(dst_width) * dst_height;
    const void* inputs[2] = {rgba, depth};
    const size_t in_bytes[2] = {ns * 16, ns * 4};
    const void* outputs[3] = {rgba_out, depth_out, source_out};
    const size_t out_bytes[3] = {nd * 16, nd * 4, nd * 4};
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 2; ++j)
            if (overlaps(outputs[i], out_bytes[i], inputs[j], in_bytes[j]))
                return fail(RAYPC_ERR_INVALID, "an output buffer overlaps an input (the warp is not in place)");
        for (int j = i + 1; j < 3; ++j)
            if (overlaps(outputs[i], out_bytes[i], outputs[j], out_bytes[j]))
                return fail(RAYPC_ERR_INVALID, "output buffers overlap");
    }
    RenderArgs cs, cd;
    std::memset(&cs, 0, sizeof(cs));
    std::memset(&cd, 0, sizeof(cd));
    int rc = camera_setup(src_cam, src_width, src_height, cs);
    if (rc) return rc;
    rc = camera_setup(dst_cam, dst_width, dst_height, cd);
    if (rc) return rc;
    std::memset(&w, 0, sizeof(w));
    auto frame = [](const RenderArgs& r, WarpCamera& c) {
        for (int k = 0; k < 3; ++k) {
            c.eye[k] = r.eye[k];
            c.fwd[k] = r.fwd[k];
            c.right[k] = r.right[k];
            c.up[k] = r.upv[k];
        }
        c.sx_scale = r.sx_scale;
        c.sy_scale = r.sy_scale;
        c.inv_w2 = r.inv_w2;
        c.inv_h2 = r.inv_h2;
        c.width = r.width;
        c.height = r.height;
    };
    frame(cs, w.src);
    frame(cd, w.dst);
    w.rgba = reinterpret_cast<const float4*>(rgba);
    w.depth = depth;
    w.n_src = static_cast<uint32_t>(ns);
    w.out = reinterpret_cast<float4*>(rgba_out);
    w.out_depth = depth_out;
    w.out_src = source_out;
    return RAYPC_OK;
}

int raypc_warp(raypc_ctx* ctx, const raypc_camera* src_cam, int src_width, int src_height, const float* rgba,
               const float* depth, const raypc_camera* dst_cam, int dst_width, int dst_height, float* rgba_out,
               float* depth_out, int32_t* source_out, void* stream) {
    WarpArgs w;
    int rc = warp_setup(ctx, src_cam, src_width, src_height, rgba, depth, dst_cam, dst_width, dst_height, rgba_out,
                        depth_out, source_out, w);
    if (rc) return rc;
    const size_t nd = static_cast<size_t>(dst_width) * dst_height;
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (nd > ctx->warp_keys_n) {
        // a warp still in flight may use the old buffers
        HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize before growing the warp buffers");
        for (int i = 0; i < 2; ++i) {
            if (ctx->warp_keys[i]) (void)hipFree(ctx->warp_keys[i]);
            ctx->warp_keys[i] = nullptr;
            ctx->warp_clean_n[i] = 0;
        }
        ctx->warp_keys_n = 0;
        for (int i = 0; i < 2; ++i) {
            if (hipMalloc(reinterpret_cast<void**>(&ctx->warp_keys[i]), nd * sizeof(unsigned long long)) != hipSuccess) {
                (void)hipGetLastError();
                for (int j = 0; j < i; ++j) {
                    (void)hipFree(ctx->warp_keys[j]);
                    ctx->warp_keys[j] = nullptr;
                }
                return fail(RAYPC_ERR_NOMEM, "warp z-buffers of %zu pixels", nd);
            }
        }
        ctx->warp_keys_n = nd;
    }
    const int cur = ctx->warp_cur, other = 1 - cur;
    w.keys = ctx->warp_keys[cur];
    w.clear_keys = ctx->warp_clean_n[cur] < nd;
    w.next_keys = ctx->warp_keys[other];
    ctx->warp_clean_n[cur] = 0;  // holds this warp's keys from now on
    ctx->warp_clean_n[other] = 0;
    HIP_TRY(launch_warp(w, static_cast<hipStream_t>(stream)), "warp kernel launches");
    ctx->warp_clean_n[other] = nd;  // emptied by this warp's resolve
    ctx->warp_cur = other;
    return RAYPC_OK;
}

int raypc_warp_noalloc(raypc_ctx* ctx, const raypc_camera* src_cam, int src_width, int src_height, const float* rgba,
                       const float* depth, const raypc_camera* dst_cam, int dst_width, int dst_height, float* rgba_out,
                       float* depth_out, int32_t* source_out, void* stream) {
    WarpArgs w;
    int rc = warp_setup(ctx, src_cam, src_width, src_height, rgba, depth, dst_cam, dst_width, dst_height, rgba_out,
                        depth_out, source_out, w);
    if (rc) return rc;
    const size_t nd = static_cast<size_t>(dst_width) * dst_height;
    if (nd > kWarpScratchPixels)
        return fail(RAYPC_ERR_INVALID, "destination of %dx%d = %zu pixels exceeds the fixed z-buffer's %zu pixels",
                    dst_width, dst_height, nd, kWarpScratchPixels);
    if (!ctx->warp_scratch) return fail(RAYPC_ERR_DEVICE, "no fixed z-buffer on device %d", ctx->device);
    DeviceGuard g(ctx->device);
    // the array keeps whatever the last call on this device left: the fill kernel empties it first
    w.keys = ctx->warp_scratch;
    w.clear_keys = 1;
    w.next_keys = nullptr;
    HIP_TRY(launch_warp(w, static_cast<hipStream_t>(stream)), "warp kernel launches");
    return RAYPC_OK;
}

int raypc_measure_peaks(raypc_ctx* ctx, double* copy_bytes_per_s, double* fma_lane_ops_per_s, void* stream) {
    if (!ctx || !copy_bytes_per_s || !fma_lane_ops_per_s) return fail(RAYPC_ERR_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    HIP_TRY(measure_peaks(copy_bytes_per_s, fma_lane_ops_per_s, static_cast<hipStream_t>(stream)),
            "peak-rate kernels");
    return RAYPC_OK;
}

int raypc_set_launch_shape(raypc_ctx* ctx, int super_log2, int tile_log2w) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    if (super_log2 < 0 || super_log2 > kMaxSuperLog2)
        return fail(RAYPC_ERR_INVALID, "super_log2 %d outside [0, %d]", super_log2, kMaxSuperLog2);
    if (tile_log2w < 0 || tile_log2w > kMaxTileLog2W)
        return fail(RAYPC_ERR_INVALID, "tile_log2w %d outside [0, %d]", tile_log2w, kMaxTileLog2W);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->super_log2 = super_log2;
    ctx->tile_log2w = tile_log2w;
    return RAYPC_OK;
}

int raypc_get_launch_shape(raypc_ctx* ctx, int* super_log2, int* tile_log2w) {
    if (!ctx || !super_log2 || !tile_log2w) return fail(RAYPC_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    *super_log2 = ctx->super_log2;
    *tile_log2w = ctx->tile_log2w;
    return RAYPC_OK;
}

int raypc_autotune_render(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                          float step, int repeats, float* times_ms, int* best_super, int* best_tile) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    if (repeats < 1 || repeats > 1000) return fail(RAYPC_ERR_INVALID, "repeats %d outside [1, 1000]", repeats);
    DeviceGuard g(ctx->device);
    const size_t bytes = static_cast<size_t>(std::max(width, 1)) * std::max(height, 1) * sizeof(float4);
    if (width < 1 || width > 16384 || height < 1 || height > 16384)
        return fail(RAYPC_ERR_INVALID, "image size %dx%d outside [1, 16384]", width, height);
    float* out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&out), bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RAYPC_ERR_NOMEM, "autotune image of %zu bytes", bytes);
    }
    constexpr int kSupers = kMaxSuperLog2 + 1, kShapes = (kMaxTileLog2W + 1) * kSupers;
    int rc = RAYPC_OK;
    float t[kShapes];
    int saved_super = kDefaultSuperLog2, saved_tile = kDefaultTileLog2W;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        saved_super = ctx->super_log2;
        saved_tile = ctx->tile_log2w;
    }
    do {
        hipError_t e = hipStreamCreate(&s);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) { rc = hip_fail(e, "autotune stream / events"); break; }
        for (int c = 0; c < kShapes && !rc; ++c) {
            {
                std::lock_guard<std::mutex> lk(ctx->mu);
                ctx->tile_log2w = c / kSupers;
                ctx->super_log2 = c % kSupers;
            }
            // one untimed render (skip state, caches), then `repeats` timed back to back
            rc = raypc_render(ctx, volume_id, cam, width, height, lod, step, out, s);
            if (!rc && (e = hipEventRecord(e0, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
            for (int r = 0; r < repeats && !rc; ++r) rc = raypc_render(ctx, volume_id, cam, width, height, lod, step, out, s);
            if (!rc && (e = hipEventRecord(e1, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
            if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
            float ms = 0.0f;
            if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = hip_fail(e, "hipEventElapsedTime");
            t[c] = ms / repeats;
        }
    } while (0);
    if (s) (void)hipStreamSynchronize(s);
    int bs = saved_super, bt = saved_tile;
    if (!rc) {
        // the default shape stays unless another is faster by more than the timing noise (1 %), so
        // that runs on one device agree on the shape
        const int def = kDefaultTileLog2W * kSupers + kDefaultSuperLog2;
        int b = def;
        for (int c = 0; c < kShapes; ++c)
            if (t[c] < t[b] && t[c] < 0.99f * t[def]) b = c;
        bt = b / kSupers;
        bs = b % kSupers;
        if (times_ms)
            for (int c = 0; c < kShapes; ++c) times_ms[c] = t[c];
        if (best_super) *best_super = bs;
        if (best_tile) *best_tile = bt;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->super_log2 = bs;  // the winner, or the previous shape when tuning failed
        ctx->tile_log2w = bt;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(out);
    return rc;
}

int raypc_render_progressive(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                             float step, int n_passes, float* const* outs, void* stream) {
    if (!ctx || !outs) return fail(RAYPC_ERR_INVALID, "NULL argument");
    if (n_passes < 1 || n_passes > 8) return fail(RAYPC_ERR_INVALID, "n_passes %d outside [1, 8]", n_passes);
    const float coarsest = std::ldexp(step, n_passes - 1);
    if (!(step >= 1.0f / 64.0f && coarsest <= 64.0f))
        return fail(RAYPC_ERR_INVALID, "pass steps %g..%g outside [1/64, 64]", coarsest, step);
    for (int k = 0; k < n_passes; ++k)
        if (!outs[k]) return fail(RAYPC_ERR_INVALID, "outs[%d] is NULL", k);
    if (lod == -1) {
        if (!cam) return fail(RAYPC_ERR_INVALID, "camera is NULL");
        const Volume* v = find_volume(ctx, volume_id);
        if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
        select_lod_impl(v, cam, height, &lod);
    }
    for (int k = 0; k < n_passes; ++k) {
        const int rc = raypc_render(ctx, volume_id, cam, width, height, lod, std::ldexp(step, n_passes - 1 - k),
                                    outs[k], stream);
        if (rc) return rc;
    }
    return RAYPC_OK;
}

int raypc_export_level(raypc_ctx* ctx, int volume_id, int lod, int field, float* out, void* stream) {
    if (!ctx || !out) return fail(RAYPC_ERR_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    int rc = check_level(v, lod);
    if (rc) return rc;
    if (field < 0 || field >= v->nf) return fail(RAYPC_ERR_INVALID, "field %d outside [0, %d)", field, v->nf);
    const Level& L = v->lv[lod];
    HIP_TRY(launch_decode(L.data[field], L.par[field], L.n, v->storage, out, 1.0f / stored_scale(v, field),
                          static_cast<hipStream_t>(stream)),
            "decode kernel launch");
    return RAYPC_OK;
}

int raypc_export_minmax(raypc_ctx* ctx, int volume_id, int lod, int field, float* out, void* stream) {
    if (!ctx || !out) return fail(RAYPC_ERR_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    int rc = check_level(v, lod);
    if (rc) return rc;
    if (field < 0 || field >= v->nf) return fail(RAYPC_ERR_INVALID, "field %d outside [0, %d)", field, v->nf);
    const Level& L = v->lv[lod];
    HIP_TRY(hipMemcpyAsync(out, L.mm[field], L.n_bricks() * sizeof(float2), hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)),
            "hipMemcpyAsync(min/max)");
    return RAYPC_OK;
}

int raypc_export_minmax_sub(raypc_ctx* ctx, int volume_id, int lod, int field, float* out, void* stream) {
    if (!ctx || !out) return fail(RAYPC_ERR_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    int rc = check_level(v, lod);
    if (rc) return rc;
    if (field < 0 || field >= v->nf) return fail(RAYPC_ERR_INVALID, "field %d outside [0, %d)", field, v->nf);
    const Level& L = v->lv[lod];
    HIP_TRY(hipMemcpyAsync(out, L.mm_sub[field], L.n_bricks() * 8 * sizeof(float2), hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)),
            "hipMemcpyAsync(sub-brick min/max)");
    return RAYPC_OK;
}

// what: 0 the skip bits (bit 10 of the flag words, packed), 1 the sub-brick flags (low bytes of the flag
// words), 2 the flag words.
static int export_skip(raypc_ctx* ctx, int volume_id, int lod, int slot, void* out, int what, void* stream) {
    if (!ctx || !out) return fail(RAYPC_ERR_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    int rc = check_level(v, lod);
    if (rc) return rc;
    if (slot < 0 || slot >= RAYPC_TF_SLOTS || !ctx->tf[slot].defined)
        return fail(RAYPC_ERR_INVALID, "transfer-function slot %d is not defined", slot);
    if (ctx->tf[slot].field >= v->nf) return fail(RAYPC_ERR_INVALID, "transfer function field outside the volume");
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = ensure_skip(ctx, v, lod, slot, s);
    if (rc) return rc;
    Level& L = v->lv[lod];
    if (what == 1)  // the low bytes of the flag words
        HIP_TRY(hipMemcpy2DAsync(out, 1, L.skip_sub, sizeof(uint16_t), 1, L.n_bricks(), hipMemcpyDeviceToDevice, s),
                "hipMemcpy2DAsync(sub-brick flags)");
    else if (what == 2)
        HIP_TRY(hipMemcpyAsync(out, L.skip_sub, L.n_bricks() * sizeof(uint16_t), hipMemcpyDeviceToDevice, s),
                "hipMemcpyAsync(skip flag words)");
    else
        HIP_TRY(launch_pack_skip_bits(L.skip_sub, L.n_bricks(), static_cast<uint32_t*>(out), s), "skip-bit packing");
    return note_skip_use(L, s);
}

int raypc_export_skiplist(raypc_ctx* ctx, int volume_id, int lod, int slot, uint32_t* out, void* stream) {
    return export_skip(ctx, volume_id, lod, slot, out, 0, stream);
}

int raypc_export_subskip(raypc_ctx* ctx, int volume_id, int lod, int slot, uint8_t* out, void* stream) {
    return export_skip(ctx, volume_id, lod, slot, out, 1, stream);
}

int raypc_export_skip_words(raypc_ctx* ctx, int volume_id, int lod, int slot, uint16_t* out, void* stream) {
    return export_skip(ctx, volume_id, lod, slot, out, 2, stream);
}

int raypc_pc_lines(raypc_ctx* ctx, int volume_id, int lod, int n_lines, const uint32_t* cells, const float* axis_lo,
                   const float* axis_hi, int n_bins, float* values, uint8_t* passes, uint32_t* hist, void* stream) {
    if (!ctx) return fail(RAYPC_ERR_INVALID, "ctx is NULL");
    DeviceGuard g(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    int rc = check_level(v, lod);
    if (rc) return rc;
    if (n_lines < 0 || n_lines > (1 << 24)) return fail(RAYPC_ERR_INVALID, "n_lines %d outside [0, 2^24]", n_lines);
    if (n_lines > 0 && !cells) return fail(RAYPC_ERR_INVALID, "cells is NULL");
    PcArgs a;
    std::memset(&a, 0, sizeof(a));
    if (hist) {
        if (n_bins < 1 || n_bins > kMaxPcBins) return fail(RAYPC_ERR_INVALID, "n_bins %d outside [1, %d]", n_bins, kMaxPcBins);
        if (!axis_lo || !axis_hi) return fail(RAYPC_ERR_INVALID, "axis_lo / axis_hi is NULL");
        for (int f = 0; f < v->nf; ++f) {
            const float w = axis_hi[f] - axis_lo[f];
            const float inv = 1.0f / w;
            if (!std::isfinite(axis_lo[f]) || !std::isfinite(axis_hi[f]) || !(w > 0.0f) || !std::isfinite(inv))
                return fail(RAYPC_ERR_INVALID, "axis %d range [%g, %g] is not a finite, non-empty interval", f,
                            static_cast<double>(axis_lo[f]), static_cast<double>(axis_hi[f]));
            a.axis_lo[f] = axis_lo[f];
            a.inv[f] = inv;
        }
    }
    const Level& L = v->lv[lod];
    for (int f = 0; f < v->nf; ++f) {
        a.field[f] = L.data[f];
        a.u8par[f] = L.par[f];
        a.active[f] = v->active[f];
        a.lo[f] = v->lo[f];
        a.hi[f] = v->hi[f];
        a.descale[f] = 1.0f / stored_scale(v, f);
    }
    a.n_fields = v->nf;
    a.storage = v->storage;
    a.coord_mask = coord_kernel_form(v->coord, a.clo, a.chi);
    a.n = L.n;
    a.nb = L.nb;
    a.n_bins = n_bins;
    a.n_lines = n_lines;
    a.cells = cells;
    a.values = values;
    a.passes = passes;
    a.hist = hist;
    HIP_TRY(launch_pc_lines(a, static_cast<hipStream_t>(stream)), "parallel-coordinates kernel launch");
    return RAYPC_OK;
}

int raypc_export_voxel_mask(raypc_ctx* ctx, int volume_id, int lod, uint8_t* out, void* stream) {
    if (!ctx || !out) return fail(RAYPC_ERR_INVALID, "NULL argument");
    DeviceGuard g(ctx->device);
    Volume* v = find_volume(ctx, volume_id);
    if (!v) return fail(RAYPC_ERR_INVALID, "unknown volume id %d", volume_id);
    int rc = check_level(v, lod);
    if (rc) return rc;
    const Level& L = v->lv[lod];
    MaskArgs a;
    std::memset(&a, 0, sizeof(a));
    int k = 0;
    for (int f = 0; f < v->nf; ++f) {
        if (!v->active[f]) continue;
        a.field[k] = L.data[f];
        a.u8par[k] = L.par[f];
        a.lo[k] = v->lo[f];
        a.hi[k] = v->hi[f];
        a.descale[k] = 1.0f / stored_scale(v, f);
        ++k;
    }
    a.n_active = k;
    a.coord_mask = coord_kernel_form(v->coord, a.clo, a.chi);
    a.n = L.n;
    a.nb = L.nb;
    a.storage = v->storage;
    a.out = out;
    HIP_TRY(launch_voxel_mask(a, static_cast<hipStream_t>(stream)), "voxel-mask kernel launch");
    return RAYPC_OK;
}

}  // extern "C"
