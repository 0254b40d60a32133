// Batches of independent cubes: one grouped launch per transform pass and
// shape class covers the tiles of every cube in the class (kernels in
// muffin_fft.hip / muffin_spectral.hip, the same per-tile code as the
// single-cube launches).  The launch descriptors live at the end of the
// batch workspace and are rebuilt whenever a cube's arrays, parameters or
// schedule change.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <algorithm>
#include <vector>

#include "muffin.h"
#include "muffin_ctx.hpp"
#include "muffin_kernels.hpp"
#include "muffin_layout.hpp"

using namespace muffin;

namespace {

enum Kind { K_ROWF = 0, K_COL = 1, K_ROWI = 2, K_SPEC = 3, K_FUSED = 4, K_NUM = 5 };

constexpr size_t kDescSlot = 256;     // device bytes reserved per (pass, cube) descriptor
static_assert(sizeof(RowDesc) <= kDescSlot && sizeof(ColDesc) <= kDescSlot &&
                  sizeof(SpecDesc) <= kDescSlot && sizeof(FusedDesc) <= kDescSlot,
              "descriptor slot too small");

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }
size_t desc_region_bytes(int n) { return align_up(size_t(K_NUM) * n * kDescSlot); }

struct Class {
    int kind;
    int key;                 // nx (row and fused passes), ny (column pass), L (spectral pass)
    int nth;                 // pixels per block of a spectral class; L of a fused class
    int variant;             // tile schedule (transform passes)
    std::vector<int> cubes;
    int nblocks;             // grid of the grouped launch
    size_t slot0;            // first descriptor slot of the class
    int lane;                // stream lane of the class (see assign_lanes)
};

// The cubes of a batch are independent: they are spread over up to
// kMaxLanes streams (lanes), balanced by voxels, and a grouped launch only
// groups cubes of one lane, so that the launches of different lanes overlap
// (the small, latency-bound launches of small cubes with the large ones).  A
// pass forks from the caller's stream to the lanes and joins back (events),
// which graph capture records as parallel branches.
constexpr int kMaxLanes = 4;

}  // namespace

struct muffin_batch {
    int n;
    int dtype;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    std::vector<muffin_ctx*> cubes;
    std::vector<Class> classes;
    std::vector<unsigned> seen;            // cube versions the descriptors describe
    std::vector<unsigned char> host_desc;  // staging copy of the descriptor region
    char* desc;                            // device descriptor region
    bool built;
    int use_graph;
    hipStream_t cap;
    hipGraphExec_t gexec;
    int passes;                            // batch passes run since setup
    int n_lanes;                           // stream lanes of the current classes
    hipStream_t lane_s[kMaxLanes];
    hipEvent_t lane_e[kMaxLanes];
    hipEvent_t fork_e;
    std::vector<int> cube_lane;            // lane of each cube's classes
};

namespace {

void drop_graph(muffin_batch* b) {
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
}

int class_of(muffin_batch* b, int kind, int key, int nth, int lane) {
    for (size_t i = 0; i < b->classes.size(); ++i) {
        const Class& c = b->classes[i];
        if (c.kind == kind && c.key == key && c.nth == nth && c.lane == lane) return int(i);
    }
    Class c{};
    c.kind = kind;
    c.key = key;
    c.nth = nth;
    c.lane = lane;
    c.variant = kind == K_COL ? kDefaultColVariant : kDefaultRowVariant;
    b->classes.push_back(c);
    return int(b->classes.size() - 1);
}

int cube_blocks(const muffin_batch* b, const Class& k, muffin_ctx* c, int variant) {
    const muffin_shape& s = c->shape;
    switch (k.kind) {
        case K_ROWF:
        case K_ROWI: return row_blocks(s.L * s.ny, s.nx, variant);
        case K_COL: return col_blocks(b->dtype, s.L, s.ny, s.nx, variant);
        case K_FUSED: return s.ny;
        default: return int((long(s.ny) * s.nx) / k.nth);
    }
}

// a class's descriptors are a packed array of its kind's struct, starting
// at byte slot0 * kDescSlot of the region
size_t desc_size(int kind) {
    if (kind == K_FUSED) return sizeof(FusedDesc);
    return kind == K_COL ? sizeof(ColDesc) : (kind == K_SPEC ? sizeof(SpecDesc) : sizeof(RowDesc));
}

// descriptor of cube c in class k; `row_out` replaces X as the inverse row
// pass's output (autotuning writes a scratch array instead)
void fill_desc(const muffin_batch* b, const Class& k, muffin_ctx* c, int first, int nblk,
               unsigned char* slot, void* row_out) {
    const muffin_shape& s = c->shape;
    if (k.kind == K_ROWF || k.kind == K_ROWI) {
        RowDesc d{};
        d.in = k.kind == K_ROWF ? (const void*)P(c, c->lay.brest) : (const void*)P(c, c->lay.z);
        d.out = k.kind == K_ROWF ? (void*)P(c, c->lay.z) : (row_out ? row_out : (void*)P(c, c->lay.x));
        d.tw = P(c, c->lay.tw);
        d.nrows = s.L * s.ny;
        d.twlog = c->twlog;
        d.first = first;
        d.nblk = nblk;
        std::memcpy(slot, &d, sizeof(d));
    } else if (k.kind == K_COL) {
        ColDesc d{};
        d.data = P(c, c->lay.z);
        d.Yf = P(c, c->lay.yf);
        d.Yfn = P(c, c->lay.yfnyq);
        d.H2 = P(c, c->lay.h2);
        d.H2nyq = P(c, c->lay.h2nyq);
        d.tw = P(c, c->lay.tw);
        d.rhoQ = rho_Q(c->params);
        d.scale = fft_scale(s);
        d.L = s.L;
        d.M = s.nx / 2;
        d.twlog = c->twlog;
        d.first = first;
        d.nblk = nblk;
        std::memcpy(slot, &d, sizeof(d));
    } else if (k.kind == K_FUSED) {
        FusedDesc d{};
        d.A.X = P(c, c->lay.x);
        d.A.zP = d.A.zPo = (char*)st(c, ST_ZP);
        d.A.zT = d.A.zTo = (char*)st(c, ST_ZT);
        d.A.zV = d.A.zVo = (char*)st(c, ST_ZV);
        d.A.GS = d.A.GSo = (char*)st(c, ST_GS);
        d.A.Z = P(c, c->lay.z);
        d.A.band_bytes = unsigned(long(s.ny) * s.nx * long(elem_size(s)));
        d.A.gshift = 0;
        d.D = P(c, c->lay.dctm);
        d.a = spec_args(c->params);
        d.tw = P(c, c->lay.tw);
        d.twlog = c->twlog;
        d.L = s.L;
        d.ny = s.ny;
        d.first = first;
        d.nblk = nblk;
        std::memcpy(slot, &d, sizeof(d));
    } else {
        SpecDesc d{};
        const long npix = long(s.ny) * s.nx;
        const unsigned bb = unsigned(npix * long(elem_size(s)));
        SpecArrays& A = d.A;
        A.X = P(c, c->lay.x);
        A.zP = A.zPo = (char*)st(c, ST_ZP);
        A.zT = A.zTo = (char*)st(c, ST_ZT);
        A.zV = A.zVo = (char*)st(c, ST_ZV);
        A.GS = A.GSo = (char*)st(c, ST_GS);
        A.Brest = P(c, c->lay.brest);
        A.band_bytes = bb;
        A.gshift = spectral_gshift(bb);
        d.D = P(c, c->lay.dctm);
        d.a = spec_args(c->params);
        d.npix = npix;
        d.Lrt = s.L;
        d.first = first;
        d.nblk = nblk;
        std::memcpy(slot, &d, sizeof(d));
    }
}

// lay out every class's blocks and write its descriptors into host_desc
void layout_class(muffin_batch* b, Class& k, int variant, void* const* row_out) {
    int next = 0;
    for (size_t j = 0; j < k.cubes.size(); ++j) {
        muffin_ctx* c = b->cubes[k.cubes[j]];
        if (k.kind == K_COL) next = (next + 31) & ~31;     // the column pass's tile order needs it
        const int nb = cube_blocks(b, k, c, variant);
        fill_desc(b, k, c, next, nb, &b->host_desc[k.slot0 * kDescSlot + j * desc_size(k.kind)],
                  row_out ? row_out[j] : nullptr);
        next += nb;
    }
    k.nblocks = next;
}

int upload(muffin_batch* b) {
    HIP_TRY(hipStreamSynchronize(b->stream));   // no launch reads the region meanwhile
    HIP_TRY(hipMemcpy(b->desc, b->host_desc.data(), b->host_desc.size(), hipMemcpyHostToDevice));
    return MUFFIN_OK;
}

// lanes: cubes of one shape and pass form stay together (they share every
// grouped launch); these groups, largest first, go to the least loaded lane
void assign_lanes(muffin_batch* b, std::vector<int>& lane_of) {
    std::vector<int> group(size_t(b->n), -1);
    std::vector<double> load;
    for (int i = 0; i < b->n; ++i) {
        if (group[size_t(i)] >= 0) continue;
        const muffin_shape& s = b->cubes[size_t(i)]->shape;
        const bool f = fused_pass(b->cubes[size_t(i)]);
        const int g = int(load.size());
        load.push_back(0.0);
        for (int j = i; j < b->n; ++j) {
            const muffin_shape& t = b->cubes[size_t(j)]->shape;
            if (group[size_t(j)] < 0 && t.nx == s.nx && t.ny == s.ny && t.L == s.L && fused_pass(b->cubes[size_t(j)]) == f) {
                group[size_t(j)] = g;
                load[size_t(g)] += double(voxels(t));
            }
        }
    }
    std::vector<int> order(load.size());
    for (size_t g = 0; g < order.size(); ++g) order[g] = int(g);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return load[size_t(x)] > load[size_t(y)]; });
    b->n_lanes = int(order.size()) < kMaxLanes ? int(order.size()) : kMaxLanes;
    std::vector<double> lane_load(size_t(b->n_lanes), 0.0);
    std::vector<int> lane_of_group(load.size(), 0);
    for (int g : order) {
        int best = 0;
        for (int l = 1; l < b->n_lanes; ++l)
            if (lane_load[size_t(l)] < lane_load[size_t(best)]) best = l;
        lane_of_group[size_t(g)] = best;
        lane_load[size_t(best)] += load[size_t(g)];
    }
    lane_of.assign(size_t(b->n), 0);
    for (int i = 0; i < b->n; ++i) lane_of[size_t(i)] = lane_of_group[size_t(group[size_t(i)])];
}

// class membership: a cube whose schedule runs the fused pass (where built)
// joins a column class and a fused class, the others the four classes of
// the three-launch pass; tile schedules chosen earlier are kept
void build_classes(muffin_batch* b) {
    std::vector<Class> old;
    old.swap(b->classes);
    std::vector<int> lane;
    assign_lanes(b, lane);
    b->cube_lane = lane;
    for (int i = 0; i < b->n; ++i) {
        const muffin_shape& s = b->cubes[i]->shape;
        const int l = lane[size_t(i)];
        if (fused_pass(b->cubes[i])) {
            b->classes[class_of(b, K_COL, s.ny, 0, l)].cubes.push_back(i);
            b->classes[class_of(b, K_FUSED, s.nx, s.L, l)].cubes.push_back(i);
        } else {
            b->classes[class_of(b, K_ROWF, s.nx, 0, l)].cubes.push_back(i);
            b->classes[class_of(b, K_COL, s.ny, 0, l)].cubes.push_back(i);
            b->classes[class_of(b, K_ROWI, s.nx, 0, l)].cubes.push_back(i);
            b->classes[class_of(b, K_SPEC, s.L, spectral_block_pixels(s.L, long(s.ny) * s.nx, int(elem_size(s))), l)]
                .cubes.push_back(i);
        }
    }
    size_t slot = 0;
    for (Class& k : b->classes) {
        k.slot0 = slot;
        slot += k.cubes.size();
        for (const Class& o : old)
            if (o.kind == k.kind && o.key == k.key && o.nth == k.nth) k.variant = o.variant;
    }
}

int rebuild(muffin_batch* b) {
    build_classes(b);
    for (Class& k : b->classes) layout_class(b, k, k.variant, nullptr);
    if (int rc = upload(b)) return rc;
    for (int i = 0; i < b->n; ++i) b->seen[i] = b->cubes[i]->version;
    b->built = true;
    drop_graph(b);
    return MUFFIN_OK;
}

bool stale(const muffin_batch* b) {
    if (!b->built) return true;
    for (int i = 0; i < b->n; ++i)
        if (b->seen[i] != b->cubes[i]->version) return true;
    return false;
}

hipError_t launch_class(const muffin_batch* b, const Class& k, int variant, hipStream_t s) {
    const size_t off = k.slot0 * kDescSlot;
    const int n = int(k.cubes.size());
    switch (k.kind) {
        case K_ROWF: return launch_row_fwd_group(b->dtype, k.key, variant, (const RowDesc*)(b->desc + off), n, k.nblocks, s);
        case K_ROWI: return launch_row_inv_group(b->dtype, k.key, variant, (const RowDesc*)(b->desc + off), n, k.nblocks, s);
        case K_COL: return launch_col_group(b->dtype, k.key, variant, (const ColDesc*)(b->desc + off), n, k.nblocks, s);
        case K_FUSED: return launch_fused_group(b->dtype, k.key, k.nth, (const FusedDesc*)(b->desc + off), n, k.nblocks, s);
        default: return launch_spectral_group(b->dtype, k.key, k.nth, (const SpecDesc*)(b->desc + off), n, k.nblocks, s);
    }
}

// the wavelet part of the pass of every cube whose W_s has wavelet bases
// (steps III and VI per basis, its terms added to B_rest), each on the
// stream of its cube's classes, after them
int dict_passes(muffin_batch* b, hipStream_t s, bool lanes) {
    for (int i = 0; i < b->n; ++i) {
        muffin_ctx* c = b->cubes[size_t(i)];
        if (c->lay.n_w == 0) continue;
        const hipStream_t keep = c->stream;
        c->stream = lanes ? b->lane_s[b->cube_lane[size_t(i)]] : s;
        const int rc = dict_pass(c);
        c->stream = keep;
        if (rc) return rc;
    }
    return MUFFIN_OK;
}

int pass_kernels(muffin_batch* b, hipStream_t s) {
    if (b->n_lanes <= 1) {
        for (int kind = 0; kind < K_NUM; ++kind)
            for (const Class& k : b->classes)
                if (k.kind == kind) HIP_TRY(launch_class(b, k, k.variant, s));
        return dict_passes(b, s, false);
    }
    for (int l = 0; l < b->n_lanes; ++l) {
        if (!b->lane_s[l]) HIP_TRY(hipStreamCreateWithFlags(&b->lane_s[l], hipStreamNonBlocking));
        if (!b->lane_e[l]) HIP_TRY(hipEventCreateWithFlags(&b->lane_e[l], hipEventDisableTiming));
    }
    if (!b->fork_e) HIP_TRY(hipEventCreateWithFlags(&b->fork_e, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(b->fork_e, s));
    for (int l = 0; l < b->n_lanes; ++l) HIP_TRY(hipStreamWaitEvent(b->lane_s[l], b->fork_e, 0));
    for (int kind = 0; kind < K_NUM; ++kind)
        for (const Class& k : b->classes)
            if (k.kind == kind) HIP_TRY(launch_class(b, k, k.variant, b->lane_s[k.lane]));
    if (int rc = dict_passes(b, s, true)) return rc;
    for (int l = 0; l < b->n_lanes; ++l) {
        HIP_TRY(hipEventRecord(b->lane_e[l], b->lane_s[l]));
        HIP_TRY(hipStreamWaitEvent(s, b->lane_e[l], 0));
    }
    return MUFFIN_OK;
}

int capture(muffin_batch* b) {
    if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? pass_kernels(b, b->cap) : MUFFIN_EDEVICE;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess || rc != MUFFIN_OK) {
        if (g) hipGraphDestroy(g);
        if (rc == MUFFIN_OK)
            set_error("batch graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        return rc == MUFFIN_OK ? MUFFIN_EDEVICE : rc;
    }
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        set_error("batch graph instantiation failed: %s", hipGetErrorString(e));
        return MUFFIN_EDEVICE;
    }
    return MUFFIN_OK;
}

// the batch of a batch context (NULL, with the error set, for anything else)
muffin_batch* batch_of(const muffin_ctx* c) {
    if (!c || !c->batch) {
        set_error("not a batch context (muffin_setup_batch)");
        return nullptr;
    }
    return c->batch;
}

int check_shapes(int n, const muffin_shape* shapes, const muffin_params* params) {
    if (n < 1 || n > MUFFIN_MAX_BATCH) {
        set_error("batch of %d cubes outside [1, %d]", n, MUFFIN_MAX_BATCH);
        return MUFFIN_EINVAL;
    }
    if (!shapes || !params) { set_error("shapes and params must be non-NULL"); return MUFFIN_EINVAL; }
    for (int i = 0; i < n; ++i) {
        if (int rc = muffin_validate(&shapes[i], &params[i])) return rc;
        if (shapes[i].L > 128) {
            set_error("cube %d: batches take band counts up to 128 (L = %d)", i, shapes[i].L);
            return MUFFIN_EUNSUPPORTED;
        }
        if (params[i].n_nu != 1 || params[i].spectral[0] != MUFFIN_DCT2_ORTHO) {
            set_error("cube %d: batches run the DCT spectral basis alone", i);
            return MUFFIN_EUNSUPPORTED;
        }
        if (shapes[i].dtype != shapes[0].dtype) {
            set_error("cube %d has dtype %d, cube 0 has %d: a batch has one dtype", i, shapes[i].dtype,
                      shapes[0].dtype);
            return MUFFIN_EINVAL;
        }
    }
    return MUFFIN_OK;
}

// Grouped launches of the three-launch pass fill the GPU differently from
// the fused pass each cube picked on its own: time `reps` real batch passes
// with the cubes' own choices and with every cube on the three-launch pass,
// each from the same saved states (restored afterwards), and keep the faster.
int choose_pass_form(muffin_batch* b, int reps) {
    std::vector<void*> saved(b->n, nullptr);
    std::vector<int> own(b->n);
    int rc = MUFFIN_OK;
    auto cleanup = [&]() {
        for (void* p : saved)
            if (p) hipFree(p);
    };
    for (int i = 0; i < b->n && rc == MUFFIN_OK; ++i) {
        muffin_ctx* c = b->cubes[i];
        own[i] = c->fused;
        if (hipMalloc(&saved[i], muffin_state_bytes(c)) != hipSuccess) {
            saved[i] = nullptr;
            set_error("batch autotune: no device memory to save cube %d's state", i);
            rc = MUFFIN_EDEVICE;
        } else {
            rc = muffin_get_state(c, saved[i]);
        }
    }
    auto set_form = [&](bool three) -> int {
        for (int i = 0; i < b->n; ++i) {
            muffin_ctx* c = b->cubes[i];
            const int sch[3] = {c->row_v, c->col_v, three ? 0 : own[i]};
            if (int r = muffin_set_schedule(c, sch)) return r;
        }
        return MUFFIN_OK;
    };
    auto restore = [&]() -> int {
        for (int i = 0; i < b->n; ++i)
            if (int r = muffin_set_state(b->cubes[i], saved[i])) return r;
        return MUFFIN_OK;
    };
    double t[2] = {0.0, 0.0};
    for (int form = 0; form < 2 && rc == MUFFIN_OK; ++form) {
        if ((rc = set_form(form == 1)) != MUFFIN_OK || (rc = restore()) != MUFFIN_OK) break;
        if ((rc = batch_iterate(b, 1)) != MUFFIN_OK) break;       // warm-up pass
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            set_error("batch autotune: event creation failed");
            rc = MUFFIN_EDEVICE;
            break;
        }
        hipError_t e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess && (rc = batch_iterate(b, reps)) != MUFFIN_OK) e = hipSuccess;
        if (rc == MUFFIN_OK && e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (rc == MUFFIN_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (rc == MUFFIN_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (rc == MUFFIN_OK && e != hipSuccess) {
            set_error("batch autotune: %s", hipGetErrorString(e));
            rc = MUFFIN_EDEVICE;
        }
        t[form] = ms;
    }
    if (rc == MUFFIN_OK) rc = set_form(t[1] < t[0]);
    if (rc == MUFFIN_OK) rc = restore();
    if (rc == MUFFIN_OK && hipStreamSynchronize(b->stream) != hipSuccess) {
        set_error("batch autotune: stream synchronisation failed");
        rc = MUFFIN_EDEVICE;
    }
    cleanup();
    return rc;
}

}  // namespace

namespace muffin {

int batch_iterate(muffin_batch* b, int n_iter) {
    if (n_iter < 0) { set_error("n_iter = %d < 0", n_iter); return MUFFIN_EINVAL; }
    if (n_iter == 0) return MUFFIN_OK;
    // a fused cube's pass starts from Z (the row spectra of B_rest), the
    // others' from B_rest (rebuilt from the state after fused passes)
    for (muffin_ctx* c : b->cubes) {
        if (fused_pass(c)) {
            if (int rc = ensure_z(c)) return rc;
        } else if (c->zvalid) {
            if (int rc = refresh_brest(c)) return rc;
        }
    }
    if (stale(b))
        if (int rc = rebuild(b)) return rc;
    for (int it = 0; it < n_iter; ++it) {
        if (b->use_graph) {
            if (!b->gexec)
                if (int rc = capture(b)) return rc;
            HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
        } else if (int rc = pass_kernels(b, b->stream)) {
            return rc;
        }
        for (muffin_ctx* c : b->cubes) {
            c->iters++;
            c->zvalid = fused_pass(c) ? 1 : 0;
        }
        b->passes++;
    }
    return MUFFIN_OK;
}

int batch_set_graph(muffin_batch* b, int enable) {
    b->use_graph = enable ? 1 : 0;
    return MUFFIN_OK;
}

int batch_iterations(const muffin_batch* b) { return b->passes; }

int batch_destroy(muffin_ctx* c) {
    muffin_batch* b = c->batch;
    if (b) {
        drop_graph(b);
        if (b->cap) hipStreamDestroy(b->cap);
        for (int l = 0; l < kMaxLanes; ++l) {
            if (b->lane_s[l]) hipStreamDestroy(b->lane_s[l]);
            if (b->lane_e[l]) hipEventDestroy(b->lane_e[l]);
        }
        if (b->fork_e) hipEventDestroy(b->fork_e);
        for (muffin_ctx* q : b->cubes) muffin_destroy(q);
        delete b;
    }
    delete c;
    return MUFFIN_OK;
}

}  // namespace muffin

extern "C" {

size_t muffin_batch_workspace_bytes(int n, const muffin_shape* shapes, const muffin_params* params) {
    if (check_shapes(n, shapes, params) != MUFFIN_OK) return 0;
    size_t total = 0;
    for (int i = 0; i < n; ++i) total += align_up(muffin_workspace_bytes(&shapes[i], &params[i]));
    return total + desc_region_bytes(n);
}

int muffin_setup_batch(muffin_ctx** out, int n, const muffin_shape* shapes, const muffin_params* params,
                       const void* const* psf, const void* const* dirty, void* workspace, size_t ws_bytes,
                       void* stream) {
    if (!out) { set_error("ctx output pointer is NULL"); return MUFFIN_EINVAL; }
    *out = nullptr;
    if (int rc = check_shapes(n, shapes, params)) return rc;
    if (!psf || !dirty || !workspace) {
        set_error("psf, dirty and workspace must be non-NULL");
        return MUFFIN_EINVAL;
    }
    const size_t need = muffin_batch_workspace_bytes(n, shapes, params);
    if (ws_bytes < need) {
        set_error("batch workspace of %zu bytes is smaller than the %zu bytes needed", ws_bytes, need);
        return MUFFIN_EWORKSPACE;
    }
    if ((reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0) {
        set_error("workspace must be %zu-byte aligned", kAlign);
        return MUFFIN_EWORKSPACE;
    }
    muffin_ctx* w = new (std::nothrow) muffin_ctx();
    muffin_batch* b = w ? new (std::nothrow) muffin_batch() : nullptr;
    if (!b) {
        delete w;
        set_error("out of host memory");
        return MUFFIN_EDEVICE;
    }
    w->batch = b;
    w->shape = shapes[0];
    w->stream = (hipStream_t)stream;
    b->n = n;
    b->dtype = shapes[0].dtype;
    b->stream = (hipStream_t)stream;
    b->ws = (char*)workspace;
    b->ws_bytes = ws_bytes;
    b->built = false;
    b->use_graph = 0;
    b->cap = nullptr;
    b->gexec = nullptr;
    b->passes = 0;
    b->n_lanes = 0;
    for (int l = 0; l < kMaxLanes; ++l) {
        b->lane_s[l] = nullptr;
        b->lane_e[l] = nullptr;
    }
    b->fork_e = nullptr;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const size_t wi = muffin_workspace_bytes(&shapes[i], &params[i]);
        muffin_ctx* c = nullptr;
        const int rc = muffin_setup(&c, &shapes[i], &params[i], psf[i], dirty[i], b->ws + off, wi, stream);
        if (rc != MUFFIN_OK) {
            batch_destroy(w);
            return rc;
        }
        b->cubes.push_back(c);
        off += align_up(wi);
    }
    b->desc = b->ws + off;
    b->host_desc.assign(desc_region_bytes(n), 0);
    b->seen.assign(n, 0);
    if (int rc = rebuild(b)) {
        batch_destroy(w);
        return rc;
    }
    *out = w;
    return MUFFIN_OK;
}

muffin_ctx* muffin_batch_cube(muffin_ctx* c, int i) {
    muffin_batch* b = batch_of(c);
    if (!b) return nullptr;
    if (i < 0 || i >= b->n) {
        set_error("cube %d outside the batch of %d", i, b->n);
        return nullptr;
    }
    return b->cubes[i];
}

int muffin_batch_autotune(muffin_ctx* ctx, int reps) {
    muffin_batch* b = batch_of(ctx);
    if (!b) return MUFFIN_EINVAL;
    if (reps < 1) { set_error("reps = %d < 1", reps); return MUFFIN_EINVAL; }
    // each cube's own schedule first (which pass form it joins), then the
    // tile schedule of every grouped transform launch
    for (muffin_ctx* c : b->cubes)
        if (int rc = muffin_autotune(c, reps, nullptr)) return rc;
    if (stale(b))
        if (int rc = rebuild(b)) return rc;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int rc = MUFFIN_OK;
    for (Class& k : b->classes) {
        if (k.kind == K_SPEC || k.kind == K_FUSED) continue;
        // the inverse row pass writes each cube's unused second state set
        std::vector<void*> scratch;
        for (int i : k.cubes) scratch.push_back(st_alt(b->cubes[i], 0));
        double best = 0.0;
        int bestv = k.variant;
        for (int v = 0; v < kNumVariants && rc == MUFFIN_OK; ++v) {
            layout_class(b, k, v, k.kind == K_ROWI ? scratch.data() : nullptr);
            if ((rc = upload(b)) != MUFFIN_OK) break;
            hipError_t e = launch_class(b, k, v, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_class(b, k, v, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                set_error("batch autotune: %s", hipGetErrorString(e));
                rc = MUFFIN_EDEVICE;
                break;
            }
            if (v == 0 || ms < best) {
                best = ms;
                bestv = v;
            }
        }
        k.variant = bestv;
        if (rc) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    // the timing used Z as scratch: a fused cube's pass restarts from B_rest
    for (muffin_ctx* c : b->cubes)
        if (fused_pass(c))
            if (int r = refresh_brest(c)) return r;
    if (int r = rebuild(b)) return r;
    return choose_pass_form(b, reps);
}

int muffin_batch_launches(const muffin_ctx* c) {
    const muffin_batch* b = batch_of(c);
    return b ? int(b->classes.size()) : -1;
}

}  // extern "C"
