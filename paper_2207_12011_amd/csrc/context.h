// context.h -- host-side state of a raypc context (internal, shared by api.hip and server.hip).
#pragma once

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/raypc.h"
#include "internal.h"

namespace raypc {

struct Server;

constexpr int kDefaultSuperLog2 = 2;  // default launch shape: super-tiles of 4 x 4 blocks (32 x 32 pixels)

// Versions of a level's skip-flag words: a brush or table change computes the flags into the next
// version, so a render still reading the previous one (on another stream) is not disturbed; a version
// is overwritten only after the renders that read it have finished (their events).
constexpr int kSkipVersions = 4;

// A stream's last use of one version of a buffer that several versions take turns in (skip flags,
// transfer-function tables): the version is overwritten only after every such event has completed.
struct StreamUse {
    hipStream_t stream;
    hipEvent_t done;  // recorded on `stream` after its last launch (or copy) that read the version
};

struct Level {
    int n = 0, nb = 0;
    void* data[kMaxFields] = {};
    float2* par[kMaxFields] = {};
    float2* mm[kMaxFields] = {};
    float2* mm_sub[kMaxFields] = {};  // per brick, its eight 4^3 sub-bricks' (min, max)
    void* rec[kMaxFields] = {};  // neighbourhood records (null when the volume keeps only the compact layout)
    uint16_t* skip_sub = nullptr; // per brick: sub-brick skip flags (bits 0-7) and empty-group bits (8, 9)
                                  // of the current version (= skip_ver[skip_cur])
    uint16_t* skip_ver[kSkipVersions] = {};
    std::vector<StreamUse> skip_users[kSkipVersions];  // launches that read each version
    int skip_cur = -1;
    bool skip_valid = false;
    uint64_t skip_brush_gen = 0, skip_tf_gen = 0;
    int skip_slot = -1;
    uint32_t n_bricks() const { return static_cast<uint32_t>(nb) * nb * nb; }
    uint32_t n_words() const { return (n_bricks() + 31) / 32; }
};

// Coordinate axes of a brush: x, y, z of the sample position and its radius.
struct CoordBrush {
    uint8_t active[4] = {};
    float lo[4] = {}, hi[4] = {};
};

struct Volume {
    int id = 0, n = 0, nf = 0, n_lods = 0, storage = 0;
    bool records = false;  // neighbourhood records kept (binary16 / float32 without RAYPC_STORAGE_COMPACT)
    float r_in = 0.55f, r_out = 1.0f;
    int f16_exp[kMaxFields] = {};  // binary16 storage: field f is stored times 2^f16_exp[f] (0 otherwise)
    Level lv[RAYPC_MAX_LODS];
    uint8_t active[kMaxFields] = {};
    float lo[kMaxFields] = {}, hi[kMaxFields] = {};
    CoordBrush coord;
    uint64_t brush_gen = 1;
    uint64_t bytes = 0;
    std::vector<void*> allocs;
    int refs = 0;  // serving requests queued or running on this volume
    // a fixed random sample of shell cells, from which each brush's field test order is chosen: their
    // values and the (min, max) of their 4^3 sub-bricks at level 0, field after field (order_k per field)
    int order_k = 0;
    std::vector<float> order_sample, order_sub_lo, order_sub_hi;
    // the last brush ordered and its order (callers hold the context mutex)
    bool order_cached = false;
    uint8_t order_active[kMaxFields] = {};
    float order_lo[kMaxFields] = {}, order_hi[kMaxFields] = {};
    int order_fields[kMaxFields] = {}, order_n = 0;
};

constexpr int kOrderSample = 2048;  // sampled shell cells per volume

// The order in which a render tests the brushed fields (brush_active / lo / hi per field of v): order[0 ..
// n_brushed) lists the active fields.  Every order gives the same image; the chosen one fetches fewer
// fields per sample on average.
void brush_order(Volume* v, const uint8_t* active, const float* lo, const float* hi, int* order, int& n_brushed);

// Versions of a slot's device table kept before one is overwritten: a new table goes to the next
// version, so renders already enqueued keep reading theirs; a version is rewritten only after the
// launches that read it (and the upload that wrote it) have finished, 256 definitions later.
constexpr int kTFVersions = 256;

// Factor by which the ray march sees field f of v: binary16 codes hold the values times 2^k.
inline float stored_scale(const Volume* v, int f) { return v->storage == kF16 ? std::ldexp(1.0f, v->f16_exp[f]) : 1.0f; }

struct TFSlot {
    bool defined = false;
    int field = 0;
    float vmin = 0, vmax = 1, ref_step = 2.0f / 256;
    float rgba[RAYPC_TF_ENTRIES * 4] = {};
    uint64_t gen = 0;
    float4* pool = nullptr;  // kTFVersions tables of RAYPC_TF_ENTRIES entries
    int version = -1;        // the current one
    float4* dev = nullptr;   // = pool + version * RAYPC_TF_ENTRIES
    std::vector<StreamUse> users[kTFVersions];  // launches and uploads that read each version
};

}  // namespace raypc

struct raypc_ctx {
    int device = 0;
    std::map<int, raypc::Volume*> vols;
    int next_id = 1;
    raypc::TFSlot tf[RAYPC_TF_SLOTS];
    uint64_t tf_gen_counter = 0;
    float ert = 0.99f;
    float bg[4] = {0, 0, 0, 0};
    bool has_bg = false;
    std::mutex mu;  // guards state shared with the serving thread
    hipStream_t upload = nullptr;  // non-blocking stream of the transfer-function uploads
    float4* tf_stage = nullptr;    // pinned staging of stream-ordered table uploads, per slot and version
    raypc::Server* server = nullptr;
    unsigned long long* warp_keys[2] = {nullptr, nullptr};  // image-warp z-buffers, used in turn, grown on demand
    size_t warp_keys_n = 0;        // capacity of each, pixels
    size_t warp_clean_n[2] = {0, 0};  // leading pixels of each known to hold the empty key
    int warp_cur = 0;              // the buffer the next warp splats into
    unsigned long long* warp_scratch = nullptr;  // this device's fixed z-buffer (raypc_warp_noalloc)
    int super_log2 = raypc::kDefaultSuperLog2;  // launch shape of single-image renders (raypc_set_launch_shape):
    int tile_log2w = raypc::kDefaultTileLog2W;  // super-tile size and wave tile shape
};


namespace raypc {
// Defined in api.hip; callers hold ctx->mu.
int set_error(int code, const char* fmt, ...);
Volume* lookup_volume(raypc_ctx* ctx, int id);
// Validate a render and fill the kernel arguments (skip list and table pointers left for the caller
// when use_volume_state is false).  Brush arrays are per field of the volume.
int prepare_render(raypc_ctx* ctx, int volume_id, const raypc_camera* cam, int width, int height, int lod,
                   float step, const uint8_t* active, const float* lo, const float* hi, const CoordBrush& coord,
                   int tf_slot, float* rgba_out, bool use_volume_state, hipStream_t s, RenderArgs& a, int& storage,
                   int& level, Volume** vol_out);
// Kernel form of a coordinate brush: the mask of enabled axes and bounds, radius as float32 squares.
uint32_t coord_kernel_form(const CoordBrush& c, float clo[4], float chi[4]);
// Skip-kernel arguments for level l of v under a brush and a transfer-function slot (out left null).
void build_skip_args(const raypc_ctx* ctx, const Volume* v, int l, const uint8_t* active, const float* lo,
                     const float* hi, const CoordBrush& coord, int tf_slot, SkipArgs& a);
}  // namespace raypc
