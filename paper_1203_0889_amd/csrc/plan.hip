// Host side of the C ABI declared in include/fmm.h: the plan object, argument
// checks, the call-order state machine and the stream-ordered pipelines
//   build_tree : bounding cube -> keys -> radix sort -> octree -> traversal -> CSR
//   upward     : P2M -> M2M
//   evaluate   : M2L + P2P -> L2L -> L2P -> outputs in input order
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>

#include "../../include/fmm.h"
#include "m2l_mfma.h"
#include "near_far.h"
#include "tree.h"

namespace fmm {

// Set for the duration of a call that must not allocate device memory
// (fmm_evaluate_noalloc): a workspace that would have to grow is an error.
thread_local bool t_no_alloc = false;

struct NoAllocError : std::logic_error {
    using std::logic_error::logic_error;
};

hipError_t DevBuf::grow(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (t_no_alloc) throw NoAllocError("a workspace of the plan is smaller than this evaluation needs");
    size_t nb = want + want / 4 + 256;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) return e;
    if (ptr) {
        hipDeviceSynchronize();
        hipFree(ptr);
    }
    ptr = p;
    bytes = nb;
    return hipSuccess;
}

hipError_t DevBuf::grow_keep(size_t want, hipStream_t s) {
    if (want <= bytes) return hipSuccess;
    if (t_no_alloc) throw NoAllocError("a workspace of the plan is smaller than this evaluation needs");
    size_t nb = want + want / 2 + 256;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) return e;
    if (ptr) {
        e = hipMemcpyAsync(p, ptr, bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipStreamSynchronize(s);
        hipFree(ptr);
    }
    ptr = p;
    bytes = nb;
    return hipSuccess;
}

// Scratch of fmm_evaluate_noalloc: a fixed device array (each GPU the
// library runs on holds its own copy until the process ends).  In host code
// `scratch` only names the symbol; its device address on a device comes from
// hipGetSymbolAddress with that device current, resolved once per device
// when a plan is created there and kept in g_scratch.
constexpr size_t kScratchBytes = (size_t)1 << 20;
constexpr size_t kScratchHeads = 256;   // bytes 0..255: the 16 claim counters of the work queue
constexpr int kScratchMaxChunks = (int)((kScratchBytes - kScratchHeads) / sizeof(double));   // energy partials
constexpr int kMaxDevices = 64;
// flag[] (16 ints, device): [0] non-finite input of a build, [1] leaf
// count, [kRefreshFlag, +1] non-finite coordinate / particle outside its
// widened leaf in a frozen-topology rebuild
constexpr int kRefreshFlag = 4;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

// The device address of `scratch` on `device` (the current device); null
// if it cannot be resolved.
void *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[device] = ptr;
        else (void)hipGetLastError();
    }
    return g_scratch[device];
}

void DevBuf::release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

}  // namespace fmm

using fmm::DevBuf;

enum { kStateCreated = 0, kStateBuilt = 1, kStateUp = 2, kStateEval = 3 };

enum Stage {
    ST_BOX = 0, ST_SORT, ST_TREE, ST_LISTS, ST_CSR, ST_P2M, ST_M2M, ST_M2L, ST_P2P, ST_L2L, ST_L2P, ST_OUT,
    ST_NF_PREP, ST_QUEUE, ST_M2L_REST, ST_NF_BUILD, ST_COUNT
};
// FP64 path: m2l, p2p.  Mixed path: nf_build (class tables, groups and
// task lists, at build time), nf_prep (bf16 multipoles, FP32 particles,
// zeroed locals), queue (the work-queue kernel: M2L and P2P tasks),
// m2l_rest (per-pair FP64 M2L of the pairs outside the class table).
static const char *kStageNames[16] = {"bbox_keys", "sort", "tree", "traverse", "csr", "p2m", "m2m", "m2l", "p2p",
                                      "l2l", "l2p", "output", "nf_prep", "queue", "m2l_rest", "nf_build"};

struct fmm_plan {
    fmm_params prm;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int state = kStateCreated;
    int64_t n = 0;
    int32_t n_inst = 0;
    std::vector<int64_t> h_off;
    std::vector<int64_t> off_on_dev;   // the offsets held by `off` (empty: none)
    // particles
    DevBuf off, ord, flag, box, scale;
    DevBuf keys, kalt, idx, valt, ikey, ialt, rank, ralt, tmp;
    DevBuf xs, ys, zs, qs, leaf_of;
    // tree
    DevBuf cb[10], crec;
    int64_t cell_cap = 0;
    DevBuf bounds, nch, counters;
    int64_t ncell = 0, nleaf = 0, nm2l = 0, np2p = 0;
    std::vector<int32_t> level_begin;  // level l cells: [level_begin[l], level_begin[l+1])
    DevBuf ppos, plist, ptmp;          // the cells with children (fmm::launch_parent_list) and its scan scratch
    // lists
    DevBuf front[2], m2l_pairs, p2p_pairs, pair_alt, m2l_ptr, m2l_src, p2p_ptr, p2p_src;
    DevBuf pair_alt2, tmp2;     // scratch of the P2P pair sort (second stream)
    int64_t cap_front = 0, cap_m2l = 0, cap_p2p = 0;
    DevBuf levdev;              // level starts of the device-driven octree build
    // second stream of fmm_build_tree: the upward pass (fmm_upward then has
    // nothing left to do) and the P2P lists, beside the traversal and the
    // M2L lists on the plan stream; up_join marks the end of its work
    hipStream_t up_side = nullptr;
    hipEvent_t up_fork = nullptr, up_join = nullptr, p2p_fork = nullptr, p2p_done = nullptr;
    bool upward_fresh = false;
    bool side_pending = false;  // the plan stream has yet to wait for up_join
    int depth_hint = 0;         // levels of the last tree
    int64_t ncell_hint = 0;     // cells of the last tree
    // expansions and fields
    DevBuf M, L, ops_m2m, ops_l2l, m2m_part;
    int ops_p = -1;
    // adjoint: transposed octant matrices and lists, duals, transposed fields
    DevBuf ops_m2m_t, ops_l2l_t, m2l_t_ptr, m2l_t_src, p2p_t_ptr, p2p_t_src, tkeys, tkeys_alt;
    DevBuf lam, mu, wts, psi_near, epsi_near, psi_far, epsi_far;
    bool adj_ready = false;
    fmm::NearFarState nf_t;
    fmm::HostReader reader;
    DevBuf phi_near, fld_near, phi_far, fld_far, echunk, epart;
    DevBuf trace, trace_count;   // task trace of the forward queue (FMM_FLAG_TRACE)
    DevBuf leaf_cost;            // P2P task durations by cell, measured by the last evaluation
    bool leaf_cost_valid = false;
    int64_t nbuild_full = 0, nbuild_kept = 0;   // builds from scratch / on a kept topology
    bool graph_step = false;     // the captured graph starts with a frozen-topology rebuild
    int32_t trace_cap = 0;
    bool traced = false;
    int32_t nechunk = 0;
    // fmm_evaluate_noalloc: the claim counters and energy partials in the
    // device's scratch array instead of the plan's buffers (null: the plan's)
    int32_t *heads_override = nullptr;
    double *epart_override = nullptr;
    fmm::NearFarState nf;
    fmm_tuning tuning;
    hipEvent_t ev_beg[ST_COUNT] = {}, ev_end[ST_COUNT] = {};
    hipEvent_t beg_of[ST_COUNT] = {};
    hipEvent_t last_ev = nullptr;
    bool ev_ok = false;
    hipEvent_t ev_early = nullptr;   // start of an early near field (queue stage begins there)
    bool early_timed = false;
    bool ev_used[ST_COUNT] = {};
    // HIP graph of the numeric part of a solve (fmm_graph_capture)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool capturing = false;
};

namespace {

fmm_status fail(fmm_plan *p, fmm_status st, const std::string &msg) {
    if (p) p->err = msg;
    return st;
}

fmm::CellArrays cells_of(fmm_plan *p) {
    fmm::CellArrays c;
    int32_t **f[10] = {&c.level, &c.ix, &c.iy, &c.iz, &c.first, &c.count, &c.child, &c.nchild, &c.parent, &c.inst};
    for (int i = 0; i < 10; i++) *f[i] = p->cb[i].as<int32_t>();
    c.rec = p->crec.as<int4>();
    return c;
}

void ensure_cells(fmm_plan *p, int64_t want) {
    if (want <= p->cell_cap) return;
    for (int i = 0; i < 10; i++) FMM_HIP_CHECK(p->cb[i].grow_keep((size_t)want * sizeof(int32_t), p->stream));
    int64_t cap = (int64_t)(p->cb[0].bytes / sizeof(int32_t));
    for (int i = 1; i < 10; i++) cap = std::min<int64_t>(cap, (int64_t)(p->cb[i].bytes / sizeof(int32_t)));
    // the records cover the same capacity (written after the tree is complete)
    FMM_HIP_CHECK(p->crec.grow((size_t)cap * sizeof(int4)));
    p->cell_cap = cap;
}

// Stage timing: record() opens a stage; mark() closes one, timed from the
// most recent event (the opening one, or the end of the previous stage).
void record(fmm_plan *p, int stage) {
    if (!p->ev_ok || p->capturing) return;
    hipEventRecord(p->ev_beg[stage], p->stream);
    p->last_ev = p->ev_beg[stage];
}

void mark(fmm_plan *p, int stage) {
    if (!p->ev_ok || !p->last_ev || p->capturing) return;
    hipEventRecord(p->ev_end[stage], p->stream);
    p->beg_of[stage] = p->last_ev;
    p->last_ev = p->ev_end[stage];
    p->ev_used[stage] = true;
}

void drop_graph(fmm_plan *p) {
    if (p->graph_exec) hipGraphExecDestroy(p->graph_exec);
    if (p->graph) hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_step = false;
}

void sync_read(fmm_plan *p, void *host, const void *dev, size_t bytes) { p->reader.read(host, dev, bytes, p->stream); }

int bits_for(int64_t n) {
    int b = 1;
    while (((int64_t)1 << b) < n) b++;
    return b;
}

bool deterministic(const fmm_plan *p) { return (p->prm.flags & FMM_FLAG_DETERMINISTIC) != 0; }
bool mutual_m2l(const fmm_plan *p) { return (p->prm.flags & FMM_FLAG_MUTUAL_M2L) != 0; }
bool mutual_p2p(const fmm_plan *p) { return (p->prm.flags & FMM_FLAG_MUTUAL_P2P) != 0; }
bool cost_reuse(const fmm_plan *p) {
    return (p->prm.flags & FMM_FLAG_COST_REUSE) && p->prm.precision == FMM_PREC_MIXED;
}

fmm::Geometry geom(fmm_plan *p) {
    fmm::Geometry g;
    g.box = p->box.as<double>();
    g.c = cells_of(p);
    return g;
}

// The parents of level l (which has a level below it) for the M2M and L2L
// launches.
fmm::LevelParents level_parents(const fmm_plan *p, int l) {
    const std::vector<int32_t> &lb = p->level_begin;
    return {p->plist.as<int32_t>(), p->ppos.as<int32_t>(), std::min(lb[l + 1] - lb[l], lb[l + 2] - lb[l + 1])};
}

fmm::NearFarArgs nf_args(fmm_plan *p);
void start_upward(fmm_plan *p);
void ensure_side(fmm_plan *p);
void start_near_early(fmm_plan *p, hipStream_t from);

void do_build(fmm_plan *p, const double *pos, const double *q) {
    hipStream_t s = p->stream;
    const int64_t n = p->n;
    const int ni = p->n_inst;
    // instance offsets and the energy chunk table on the device: copied only
    // when they differ from the last build's (a copy from pageable host
    // memory waits for the stream, which would idle the GPU between steps)
    const size_t off_bytes = p->off.bytes;
    FMM_HIP_CHECK(p->off.grow((ni + 1) * sizeof(int64_t)));
    if (p->off.bytes != off_bytes) p->off_on_dev.clear();
    const bool new_off = p->off_on_dev != p->h_off;
    if (new_off) {
        FMM_HIP_CHECK(hipMemcpyAsync(p->off.ptr, p->h_off.data(), (ni + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
        p->off_on_dev.clear();   // valid once the chunk table is copied too
    }
    FMM_HIP_CHECK(p->ord.grow(6 * ni * sizeof(unsigned long long)));
    FMM_HIP_CHECK(p->flag.grow(16 * sizeof(int)));
    FMM_HIP_CHECK(p->box.grow(4 * ni * sizeof(double)));
    FMM_HIP_CHECK(p->scale.grow(ni * sizeof(double)));
    FMM_HIP_CHECK(hipMemsetAsync(p->flag.ptr, 0, 16 * sizeof(int), s));
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    FMM_HIP_CHECK(p->keys.grow(nn * 8));
    FMM_HIP_CHECK(p->kalt.grow(nn * 8));
    FMM_HIP_CHECK(p->idx.grow(nn * 4));
    FMM_HIP_CHECK(p->valt.grow(nn * 4));
    FMM_HIP_CHECK(p->xs.grow(nn * 8));
    FMM_HIP_CHECK(p->ys.grow(nn * 8));
    FMM_HIP_CHECK(p->zs.grow(nn * 8));
    FMM_HIP_CHECK(p->qs.grow(nn * 8));
    FMM_HIP_CHECK(p->leaf_of.grow(nn * 4));
    FMM_HIP_CHECK(p->tmp.grow(std::max(fmm::radix_tmp_elems(n), fmm::scan_tmp_elems(n)) * sizeof(int32_t)));
    if (ni > 1) {
        FMM_HIP_CHECK(p->ikey.grow(nn * 4));
        FMM_HIP_CHECK(p->ialt.grow(nn * 4));
        FMM_HIP_CHECK(p->rank.grow(nn * 4));
        FMM_HIP_CHECK(p->ralt.grow(nn * 4));
    }
    if (new_off) {
        std::vector<int32_t> co = fmm::energy_chunks(p->h_off);
        p->nechunk = co.back();
        FMM_HIP_CHECK(p->echunk.grow(co.size() * 4));
        FMM_HIP_CHECK(p->epart.grow((size_t)std::max(p->nechunk, 1) * 8));
        FMM_HIP_CHECK(hipMemcpyAsync(p->echunk.ptr, co.data(), co.size() * 4, hipMemcpyHostToDevice, s));
        p->off_on_dev = p->h_off;
    }
    const double *pbox = p->prm.box_min;
    double ubox[4] = {pbox[0], pbox[1], pbox[2], p->prm.box_side};
    bool user = (p->prm.flags & FMM_FLAG_USER_BOX) != 0;

    record(p, ST_BOX);
    fmm::launch_bbox(pos, n, p->off.as<int64_t>(), ni, p->ord.as<unsigned long long>(), p->flag.as<int>(), s);
    fmm::launch_box_finish(p->ord.as<unsigned long long>(), ni, p->off.as<int64_t>(), user, ubox, p->box.as<double>(),
                           p->scale.as<double>(), s);
    fmm::launch_keys(pos, n, p->off.as<int64_t>(), ni, p->box.as<double>(), p->scale.as<double>(),
                     p->keys.as<uint64_t>(), p->idx.as<uint32_t>(), s);
    mark(p, ST_BOX);
    fmm::radix_sort_u64(p->keys.as<uint64_t>(), p->idx.as<uint32_t>(), p->kalt.as<uint64_t>(), p->valt.as<uint32_t>(), n,
                        0, 63, p->tmp.as<int32_t>(), s);
    fmm::sort_by_instance(p->keys.as<uint64_t>(), p->idx.as<uint32_t>(), p->kalt.as<uint64_t>(), p->valt.as<uint32_t>(),
                          p->ikey.as<uint32_t>(), p->ialt.as<uint32_t>(), p->rank.as<uint32_t>(),
                          p->ralt.as<uint32_t>(), n, p->off.as<int64_t>(), ni, p->tmp.as<int32_t>(), s);
    fmm::launch_gather(pos, q, p->idx.as<uint32_t>(), n, p->xs.as<double>(), p->ys.as<double>(), p->zs.as<double>(),
                       p->qs.as<double>(), s);
    mark(p, ST_SORT);

    // ---- octree, level by level on the device: batches of levels are
    // enqueued with their sizes kept on the device, and one host read per
    // batch returns the level starts (a tree larger than the cell capacity
    // is rebuilt with more).
    ensure_cells(p, std::max<int64_t>({2 * ni, n / std::max(1, p->prm.ncrit) * 3 + 64, p->ncell_hint}));
    const int nlev = p->prm.max_level + 3;
    FMM_HIP_CHECK(p->levdev.grow((size_t)(nlev + 1) * sizeof(int32_t)));
    int32_t *lev = p->levdev.as<int32_t>();
    std::vector<int32_t> hl(nlev + 1);
    int32_t le = ni;
    for (int attempt = 0;; attempt++) {
        const int32_t cap = (int32_t)std::min<int64_t>(p->cell_cap, ((int64_t)1 << 31) - 1);
        FMM_HIP_CHECK(p->bounds.grow((size_t)cap * 9 * sizeof(int32_t)));
        FMM_HIP_CHECK(p->nch.grow((size_t)(cap + 1) * sizeof(int32_t) * 2 + 64));
        int32_t *nch = p->nch.as<int32_t>();
        int32_t *csum = nch + (cap + 1);
        int32_t *total = csum + (cap + 1);
        fmm::launch_roots(p->off.as<int64_t>(), ni, cells_of(p), s);
        fmm::launch_tree_levels_init(lev, ni, nlev, s);
        // levels 0 .. max_level - 1 can have children; the depth of the
        // last tree (or of a uniform one) sets the first batch
        int level = 0;
        int batch = p->depth_hint > 0 ? p->depth_hint + 1 : 2;
        if (p->depth_hint <= 0)
            for (int64_t m = std::max(1, p->prm.ncrit); m < n; m *= 8) batch++;
        bool over = false;
        for (;;) {
            const int stop = std::min(level + batch, p->prm.max_level);
            for (; level < stop; level++)
                fmm::launch_tree_level_dev(cells_of(p), lev, level, nlev, p->prm.ncrit, p->prm.max_level,
                                           p->keys.as<uint64_t>(), p->bounds.as<int32_t>(), nch, csum, total, cap,
                                           s);
            sync_read(p, hl.data(), lev, (size_t)(nlev + 1) * sizeof(int32_t));
            if (hl[nlev]) {
                over = true;
                break;
            }
            if (level >= p->prm.max_level || hl[level + 1] == hl[level]) break;   // the last level had no children
            batch = 2;
        }
        if (!over) break;
        if (attempt > 8) throw std::runtime_error("octree: cell capacity did not converge");
        ensure_cells(p, (int64_t)p->cell_cap * 2);
    }
    p->level_begin.assign(1, 0);
    for (int l = 1; l < nlev && hl[l] > hl[l - 1]; l++) p->level_begin.push_back(hl[l]);
    le = p->level_begin.back();
    p->depth_hint = (int)p->level_begin.size() - 1;
    p->ncell_hint = le;
    p->ncell = le;
    if ((size_t)p->ncell * sizeof(int4) > p->crec.bytes) throw std::runtime_error("cell records smaller than the tree");
    fmm::launch_leaf_of(cells_of(p), (int32_t)p->ncell, p->leaf_of.as<int32_t>(), p->flag.as<int32_t>() + 1, s);
    mark(p, ST_TREE);
    // work on the second stream (the P2P lists, the upward pass): this
    // stream waits for it when the build returns (or throws)
    struct JoinSide {
        fmm_plan *p;
        ~JoinSide() {
            if (p->side_pending) (void)hipStreamWaitEvent(p->stream, p->up_join, 0);
            p->side_pending = false;
        }
    } join_side{p};

    // the parents of every level for the level-by-level M2M and L2L, on the
    // second stream beside the traversal (its later work, the upward pass
    // included, follows on that stream; this stream joins it at the end).
    // The fork is marked here; its launches are enqueued once the
    // traversal's are, so that the host enqueues them while the GPU
    // traverses instead of the GPU waiting for the host.
    FMM_HIP_CHECK(p->ppos.grow(((size_t)p->ncell + 1) * sizeof(int32_t)));
    FMM_HIP_CHECK(p->plist.grow((size_t)std::max<int64_t>(p->ncell, 1) * sizeof(int32_t)));
    FMM_HIP_CHECK(p->ptmp.grow(fmm::scan_tmp_elems(p->ncell) * sizeof(int32_t)));
    ensure_side(p);
    FMM_HIP_CHECK(hipEventRecord(p->p2p_fork, s));
    bool parents_listed = false;

    // the non-finite flag and the leaf count are read back with the
    // traversal's sizes (the traversal runs on any tree, even one built from
    // non-finite coordinates, which is then rejected)
    // ---- dual tree traversal, breadth first: every step is enqueued at once
    // (sizes stay on the device); one read-back checks capacities and the
    // whole traversal is rerun with larger buffers if any overflowed.
    const int64_t ncell = p->ncell;
    const int bits = bits_for(ncell);
    const bool key32 = 2 * bits <= 32;
    const size_t ksz = key32 ? 4 : 8;
    const int nlevels = (int)p->level_begin.size() - 1;
    const int nsteps = 2 * nlevels + 1;
    if (p->cap_front < 1024) p->cap_front = std::max<int64_t>(4096, 8 * ncell);
    p->cap_front = std::max<int64_t>(p->cap_front, 2 * (int64_t)ni);
    if (p->cap_m2l < 1024) p->cap_m2l = std::max<int64_t>(4096, 64 * ncell);
    if (p->cap_p2p < 1024) p->cap_p2p = std::max<int64_t>(4096, 32 * ncell);
    FMM_HIP_CHECK(p->counters.grow((size_t)(nsteps + 6) * sizeof(int32_t)));
    int32_t *ctr = p->counters.as<int32_t>();
    std::vector<int32_t> hc(nsteps + 5);
    const uint32_t ta = (uint32_t)p->prm.theta_num, tb = (uint32_t)p->prm.theta_den;
    for (int attempt = 0;; attempt++) {
        FMM_HIP_CHECK(p->front[0].grow(p->cap_front * sizeof(int2)));
        FMM_HIP_CHECK(p->front[1].grow(p->cap_front * sizeof(int2)));
        FMM_HIP_CHECK(p->m2l_pairs.grow(p->cap_m2l * ksz));
        FMM_HIP_CHECK(p->p2p_pairs.grow(p->cap_p2p * ksz));
        FMM_HIP_CHECK(hipMemsetAsync(ctr, 0, (size_t)(nsteps + 3) * sizeof(int32_t), s));
        fmm::launch_init_frontier(p->off.as<int64_t>(), ni, p->front[0].as<int2>(), ctr, s);
        fmm::PairBuf pb{p->m2l_pairs.ptr, p->p2p_pairs.ptr, (int32_t)p->cap_m2l, (int32_t)p->cap_p2p, key32};
        for (int k = 0; k < nsteps; k++)
            fmm::launch_traverse(cells_of(p), p->front[k & 1].as<int2>(), ctr + 2 + k, p->front[(k + 1) & 1].as<int2>(),
                                 ctr + 3 + k, (int32_t)p->cap_front, pb, ctr, bits, ta, tb, s);
        FMM_HIP_CHECK(hipMemcpyAsync(ctr + nsteps + 3, p->flag.ptr, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (!parents_listed) {
            FMM_HIP_CHECK(hipStreamWaitEvent(p->up_side, p->p2p_fork, 0));
            p->side_pending = true;
            fmm::launch_parent_list(cells_of(p), (int32_t)p->ncell, p->ppos.as<int32_t>(), p->plist.as<int32_t>(),
                                    p->ptmp.as<int32_t>(), p->up_side);
            FMM_HIP_CHECK(hipEventRecord(p->up_join, p->up_side));
            parents_listed = true;
        }
        sync_read(p, hc.data(), ctr, (size_t)(nsteps + 5) * sizeof(int32_t));
        if (hc[nsteps + 3]) throw std::invalid_argument("non-finite particle coordinate");
        p->nleaf = hc[nsteps + 4];
        int64_t fmax = *std::max_element(hc.begin() + 2, hc.begin() + nsteps + 3);
        bool over = false;
        if (fmax > p->cap_front) {
            p->cap_front = fmax + fmax / 2;
            over = true;
        }
        if (hc[0] > p->cap_m2l) {
            p->cap_m2l = (int64_t)hc[0] + hc[0] / 4;
            over = true;
        }
        if (hc[1] > p->cap_p2p) {
            p->cap_p2p = (int64_t)hc[1] + hc[1] / 4;
            over = true;
        }
        if (!over) break;
        if (attempt > 4) throw std::runtime_error("traversal capacity did not converge");
    }
    if (hc[nsteps + 2] != 0) throw std::runtime_error("traversal did not terminate in the expected number of steps");
    p->nm2l = hc[0];
    p->np2p = hc[1];
    mark(p, ST_LISTS);

    // ---- CSR lists grouped by target.  Only the target bits are sorted:
    // every consumer is indifferent to the order of a target's sources
    // (classes are deduplicated per group, the FP64 path and the queue add
    // with atomics or in FP32), and fmm_copy_lists sorts each target's
    // sources when it returns the canonical (target, source) order.
    int64_t mx = std::max<int64_t>(std::max(p->nm2l, p->np2p), 1);
    FMM_HIP_CHECK(p->pair_alt.grow(mx * ksz));
    FMM_HIP_CHECK(p->tmp.grow(std::max(p->tmp.bytes, fmm::radix_tmp_elems(mx) * sizeof(int32_t))));
    FMM_HIP_CHECK(p->m2l_ptr.grow((ncell + 1) * 4));
    FMM_HIP_CHECK(p->p2p_ptr.grow((ncell + 1) * 4));
    FMM_HIP_CHECK(p->m2l_src.grow(std::max<int64_t>(p->nm2l, 1) * 4));
    FMM_HIP_CHECK(p->p2p_src.grow(std::max<int64_t>(p->np2p, 1) * 4));
    // the P2P list (and, mixed, its leaf order) on the second stream with
    // scratch of its own, the M2L list here
    FMM_HIP_CHECK(p->pair_alt2.grow(std::max<int64_t>(p->np2p, 1) * ksz));
    FMM_HIP_CHECK(p->tmp2.grow(fmm::radix_tmp_elems(std::max<int64_t>(p->np2p, 1)) * sizeof(int32_t)));
    ensure_side(p);
    FMM_HIP_CHECK(hipEventRecord(p->p2p_fork, s));
    FMM_HIP_CHECK(hipStreamWaitEvent(p->up_side, p->p2p_fork, 0));
    p->side_pending = true;
    void *lists[2] = {p->m2l_pairs.ptr, p->p2p_pairs.ptr};
    void *alts[2] = {p->pair_alt.ptr, p->pair_alt2.ptr};
    int32_t *tmps[2] = {p->tmp.as<int32_t>(), p->tmp2.as<int32_t>()};
    int64_t cnts[2] = {p->nm2l, p->np2p};
    int32_t *ptrs[2] = {p->m2l_ptr.as<int32_t>(), p->p2p_ptr.as<int32_t>()};
    int32_t *srcs[2] = {p->m2l_src.as<int32_t>(), p->p2p_src.as<int32_t>()};
    hipStream_t on[2] = {s, p->up_side};
    for (int t = 0; t < 2; t++) {   // the M2L sort (the longer chain) is enqueued first
        bool in_alt = false;   // an odd number of passes leaves the sorted pairs in the scratch buffer
        // deterministic or mutual: the whole key (target, source), so that
        // each target's sources come in ascending order whatever order the
        // traversal appended them in; otherwise only the target bits
        const int lo_bit = deterministic(p) || mutual_m2l(p) || mutual_p2p(p) ? 0 : bits;
        if (key32)
            fmm::radix_sort_u32((uint32_t *)lists[t], nullptr, (uint32_t *)alts[t], nullptr, cnts[t], lo_bit,
                                2 * bits, tmps[t], on[t], &in_alt);
        else
            fmm::radix_sort_u64((uint64_t *)lists[t], nullptr, (uint64_t *)alts[t], nullptr, cnts[t], lo_bit,
                                2 * bits, tmps[t], on[t], &in_alt);
        fmm::launch_csr(in_alt ? alts[t] : lists[t], key32, cnts[t], bits, (int32_t)ncell, ptrs[t], srcs[t], on[t]);
        if (t == 1) {
            if (p->prm.precision == FMM_PREC_MIXED) {
                fmm::build_p2p_leaves(p->nf, nf_args(p), p->up_side);
                // the near field needs nothing more: it runs beside the
                // upward pass and the far-field build
                start_near_early(p, p->up_side);
            }
            FMM_HIP_CHECK(hipEventRecord(p->p2p_done, p->up_side));
            FMM_HIP_CHECK(hipEventRecord(p->up_join, p->up_side));
        }
    }
    mark(p, ST_CSR);

    // the upward pass needs only the tree; started here it runs beside the
    // near/far build (started before the traversal it slowed the traversal
    // by more than it saved; started after the build's per-pair class pass
    // it gained nothing measurable)
    if (n > 0) start_upward(p);
    if (p->prm.precision == FMM_PREC_MIXED) {
        fmm::NearFarArgs a = nf_args(p);
        a.p2p_ready = p->p2p_done;   // the P2P leaf order, built on the second stream
        fmm::build_near_far_mixed(p->nf, a, s);
        mark(p, ST_NF_BUILD);
    } else if (fmm::m2l_f64_supported(p->prm.p) && !mutual_m2l(p)) {
        // the FP64 path's M2L runs over the same class tables, on the FP64
        // matrix cores (the mutual M2L runs per pair)
        fmm::build_near_far_mixed(p->nf, nf_args(p), s);
        mark(p, ST_NF_BUILD);
    }
}

fmm::NearFarArgs nf_args(fmm_plan *p) {
    fmm::NearFarArgs a;
    a.g = geom(p);
    a.ncell = (int32_t)p->ncell;
    a.nleaf = p->nleaf;
    a.n = p->n;
    a.nm2l = p->nm2l;
    a.p = p->prm.p;
    a.m2l_ptr = p->m2l_ptr.as<int32_t>();
    a.m2l_src = p->m2l_src.as<int32_t>();
    a.p2p_ptr = p->p2p_ptr.as<int32_t>();
    a.p2p_src = p->p2p_src.as<int32_t>();
    a.leaf_of = p->leaf_of.as<int32_t>();
    a.xs = p->xs.as<double>();
    a.ys = p->ys.as<double>();
    a.zs = p->zs.as<double>();
    a.qs = p->qs.as<double>();
    a.M = p->M.as<double>();
    a.L = p->L.as<double>();
    a.phi = p->phi_near.as<double>();
    a.fld = p->fld_near.as<double>();
    a.tuning = p->tuning;
    a.reader = &p->reader;
    a.deterministic = deterministic(p);
    a.f64 = p->prm.precision == FMM_PREC_FP64;
    return a;
}

void ensure_ops(fmm_plan *p) {
    int pp = p->prm.p;
    if (p->ops_p == pp) return;
    const int P = fmm::ncoef(pp);
    std::vector<double> a = fmm::build_translation_ops(pp, 0), b = fmm::build_translation_ops(pp, 1);
    std::vector<double> at = fmm::transpose_ops(a, pp), bt = fmm::transpose_ops(b, pp);
    FMM_HIP_CHECK(p->ops_m2m.grow(a.size() * 8));
    FMM_HIP_CHECK(p->ops_l2l.grow(b.size() * 8));
    FMM_HIP_CHECK(p->ops_m2m_t.grow(at.size() * 8));
    FMM_HIP_CHECK(p->ops_l2l_t.grow(bt.size() * 8));
    FMM_HIP_CHECK(hipMemcpy(p->ops_m2m.ptr, a.data(), a.size() * 8, hipMemcpyHostToDevice));
    FMM_HIP_CHECK(hipMemcpy(p->ops_l2l.ptr, b.data(), b.size() * 8, hipMemcpyHostToDevice));
    FMM_HIP_CHECK(hipMemcpy(p->ops_m2m_t.ptr, at.data(), at.size() * 8, hipMemcpyHostToDevice));
    FMM_HIP_CHECK(hipMemcpy(p->ops_l2l_t.ptr, bt.data(), bt.size() * 8, hipMemcpyHostToDevice));
    (void)P;
    p->ops_p = pp;
}

// P2M and M2M on stream s; with `side` the stage events are recorded on s
// directly (it is not the plan's stream).
void upward_kernels(fmm_plan *p, hipStream_t s, bool side) {
    const int P = fmm::ncoef(p->prm.p);
    ensure_ops(p);
    FMM_HIP_CHECK(p->M.grow((size_t)std::max<int64_t>(p->ncell, 1) * P * 8));
    int depth = (int)p->level_begin.size() - 1;  // number of levels present
    int32_t widest = 1;
    for (int l = 0; l + 1 < depth; l++) widest = std::max(widest, level_parents(p, l).npar_max);
    FMM_HIP_CHECK(p->m2m_part.grow((size_t)8 * widest * P * 8));
    fmm::Geometry g = geom(p);
    const bool timed = side && p->ev_ok && !p->capturing;
    if (timed) FMM_HIP_CHECK(hipEventRecord(p->ev_beg[ST_P2M], s));
    else record(p, ST_P2M);
    fmm::launch_p2m(g, (int32_t)p->ncell, p->prm.p, p->xs.as<double>(), p->ys.as<double>(), p->zs.as<double>(),
                    p->qs.as<double>(), p->M.as<double>(), s);
    if (timed) FMM_HIP_CHECK(hipEventRecord(p->ev_end[ST_P2M], s));
    else mark(p, ST_P2M);
    for (int l = depth - 2; l >= 0; l--)
        fmm::launch_m2m_level(g, p->level_begin[l], p->level_begin[l + 1], p->prm.p, level_parents(p, l),
                              p->ops_m2m.as<double>(), p->M.as<double>(), p->m2m_part.as<double>(), s);
    if (timed) {
        FMM_HIP_CHECK(hipEventRecord(p->ev_end[ST_M2M], s));
        p->beg_of[ST_P2M] = p->ev_beg[ST_P2M];
        p->beg_of[ST_M2M] = p->ev_end[ST_P2M];
        p->ev_used[ST_P2M] = p->ev_used[ST_M2M] = true;
    } else {
        mark(p, ST_M2M);
    }
}

void do_upward(fmm_plan *p) {
    if (p->upward_fresh && !p->capturing) {   // done by fmm_build_tree, nothing changed since
        p->upward_fresh = false;
        return;
    }
    p->upward_fresh = false;
    upward_kernels(p, p->stream, false);
}

// The upward pass needs only the sorted particles and the tree, so a full
// build starts it on a second stream (default priority) before the
// near/far build and joins it back at the end of the build.
void ensure_side(fmm_plan *p) {
    if (p->up_side) return;
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&p->up_side, hipStreamNonBlocking));   // default priority
    FMM_HIP_CHECK(hipEventCreateWithFlags(&p->up_fork, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&p->up_join, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&p->p2p_fork, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&p->p2p_done, hipEventDisableTiming));
}

void start_upward(fmm_plan *p) {
    ensure_side(p);
    FMM_HIP_CHECK(hipEventRecord(p->up_fork, p->stream));
    FMM_HIP_CHECK(hipStreamWaitEvent(p->up_side, p->up_fork, 0));
    p->side_pending = true;
    upward_kernels(p, p->up_side, true);
    FMM_HIP_CHECK(hipEventRecord(p->up_join, p->up_side));
    p->upward_fresh = true;
}

// The mixed path's near field (P2P tasks of the work queue) depends only on
// the particles, the tree and the P2P lists (Sec. 3: a task runs once its
// inputs exist): started here, on `from`, it runs beside the upward pass
// and the far-field build, and the next evaluation's queue joins it.  Not
// with a task trace (its buffers are sized by the evaluation).
void ensure_eval_buffers(fmm_plan *p);
void start_near_early(fmm_plan *p, hipStream_t from) {
    if (p->prm.precision != FMM_PREC_MIXED || (p->prm.flags & FMM_FLAG_TRACE) || p->n == 0 ||
        p->tuning.early_p2p_per_cu <= 0 || p->tuning.p2p_per_cu <= 0)
        return;
    ensure_eval_buffers(p);
    fmm::NearFarArgs a = nf_args(p);
    if (cost_reuse(p)) {
        FMM_HIP_CHECK(p->leaf_cost.grow((size_t)std::max<int64_t>(p->ncell, 1) * sizeof(float)));
        a.cost_out = p->leaf_cost.as<float>();
    }
    const bool timed = p->ev_ok && !p->capturing;
    if (timed) FMM_HIP_CHECK(hipEventRecord(p->ev_early, from));
    const bool started = fmm::near_far_start_p2p(p->nf, a, from);
    p->early_timed = started && timed;
    if (started && cost_reuse(p)) p->leaf_cost_valid = true;
}

// Workspaces of the evaluate stage (locals, near and far fields).
void ensure_eval_buffers(fmm_plan *p) {
    const int P = fmm::ncoef(p->prm.p);
    const size_t nn = (size_t)std::max<int64_t>(p->n, 1);
    FMM_HIP_CHECK(p->L.grow((size_t)std::max<int64_t>(p->ncell, 1) * P * 8));
    FMM_HIP_CHECK(p->phi_near.grow(nn * 8));
    FMM_HIP_CHECK(p->fld_near.grow(nn * 24));
    FMM_HIP_CHECK(p->phi_far.grow(nn * 8));
    FMM_HIP_CHECK(p->fld_far.grow(nn * 24));
}

void do_evaluate(fmm_plan *p, double *phi, double *field, double *force, double *energy) {
    hipStream_t s = p->stream;
    ensure_eval_buffers(p);
    fmm::Geometry g = geom(p);
    const int32_t ncell = (int32_t)p->ncell;
    bool deferred = false;   // the queue's P2P tail still runs on the second stream
    // if anything below throws while the tail runs, the plan's stream still
    // waits for it: later work on this stream (the next evaluation's
    // zeroing of the claim counters and rewrite of the FP32 particles, a
    // release of the plan) must not overlap it
    struct DeferredJoin {
        fmm_plan *p;
        bool pending = false;
        ~DeferredJoin() {
            if (!pending) return;
            fmm::NearFarState &nf = p->nf;
            if (nf.tail_pending && nf.side && nf.after_side) {   // the tail was never launched
                (void)hipEventRecord(nf.after_side, nf.side);
                (void)hipStreamWaitEvent(p->stream, nf.after_side, 0);
                if (nf.tail_early && nf.side3 && nf.early_done) {
                    (void)hipEventRecord(nf.early_done, nf.side3);
                    (void)hipStreamWaitEvent(p->stream, nf.early_done, 0);
                }
                nf.tail_pending = false;
            } else if (nf.join) {
                (void)hipStreamWaitEvent(p->stream, nf.join, 0);
            }
        }
    } join_guard{p};
    fmm::NearFarArgs a_nf;   // the mixed path's arguments (the P2P tail needs them again)
    bool time_queue = false;  // the queue stage ends at the join (recorded after the tail)
    record(p, ST_M2L);
    if (p->prm.precision == FMM_PREC_FP64) {
        if (mutual_m2l(p))
            fmm::launch_m2l_fp64_mutual(g, ncell, p->prm.p, p->m2l_ptr.as<int32_t>(), p->m2l_src.as<int32_t>(),
                                        p->nm2l, p->M.as<double>(), p->L.as<double>(), s);
        else if (p->nf.built && p->nf.f64)
            fmm::m2l_f64_run(p->nf, nf_args(p), s);
        else
            fmm::launch_m2l_fp64(g, ncell, p->prm.p, p->m2l_ptr.as<int32_t>(), p->m2l_src.as<int32_t>(), p->nm2l,
                                 p->M.as<double>(), p->L.as<double>(), deterministic(p), s);
        mark(p, ST_M2L);
        if (mutual_p2p(p))
            fmm::launch_p2p_fp64_mutual(g, ncell, p->n, p->p2p_ptr.as<int32_t>(), p->p2p_src.as<int32_t>(),
                                        p->xs.as<double>(), p->ys.as<double>(), p->zs.as<double>(),
                                        p->qs.as<double>(), p->phi_near.as<double>(), p->fld_near.as<double>(), s);
        else
            fmm::launch_p2p_fp64(g, ncell, p->p2p_ptr.as<int32_t>(), p->p2p_src.as<int32_t>(), p->xs.as<double>(),
                                 p->ys.as<double>(), p->zs.as<double>(), p->qs.as<double>(), p->phi_near.as<double>(),
                                 p->fld_near.as<double>(), s);
        mark(p, ST_P2P);
    } else {
        a_nf = nf_args(p);
        a_nf.heads = p->heads_override;
        fmm::NearFarArgs &a = a_nf;
        if (p->prm.flags & FMM_FLAG_TRACE) {
            // one record per task: M2L tasks plus target leaves
            const int64_t cap = (int64_t)p->nf.ntask + p->nleaf;
            FMM_HIP_CHECK(p->trace.grow((size_t)std::max<int64_t>(cap, 1) * sizeof(fmm_task_record)));
            FMM_HIP_CHECK(p->trace_count.grow(sizeof(int32_t)));
            p->trace_cap = (int32_t)cap;
            a.trace = p->trace.as<fmm_task_record>();
            a.trace_count = p->trace_count.as<int32_t>();
            a.trace_cap = p->trace_cap;
            p->traced = true;
        }
        // the queue measures every P2P task for the next kept-topology
        // rebuild (leaf_cost is sized by the build)
        if (cost_reuse(p)) {
            a.cost_out = p->leaf_cost.as<float>();
            p->leaf_cost_valid = true;
        }
        fmm::near_far_prepare(p->nf, a, s);
        mark(p, ST_NF_PREP);
        // with a P2P side kernel the P2P tasks run on beside the FP64 M2L
        // rest, L2L and L2P, joined by more P2P workgroups once those are
        // queued; the near field is joined before the outputs
        join_guard.pending = true;   // also if the launch itself throws half way
        bool joined_early = false;
        deferred = fmm::near_far_queue(p->nf, a, s, /*defer_join=*/true, &joined_early);
        join_guard.pending = deferred;
        // with an early near field the queue stage begins where it started
        hipEvent_t q_beg = joined_early ? (p->early_timed ? p->ev_early : nullptr) : p->last_ev;
        p->early_timed = false;
        if (!deferred) {
            if (q_beg && p->ev_ok && !p->capturing) {
                hipEventRecord(p->ev_end[ST_QUEUE], s);
                p->beg_of[ST_QUEUE] = q_beg;
                p->ev_used[ST_QUEUE] = true;
                p->last_ev = p->ev_end[ST_QUEUE];
            }
        } else if (p->ev_ok && !p->capturing && q_beg) {
            // the queue stage ends with all its kernels (the join, on the side
            // stream, recorded after the tail); the next stage begins after
            // k_queue and the sum of its partials
            p->beg_of[ST_QUEUE] = q_beg;
            time_queue = true;
            record(p, ST_M2L_REST);
        }
        fmm::near_far_rest(p->nf, a, s);
        mark(p, ST_M2L_REST);
    }
    int depth = (int)p->level_begin.size() - 1;
    for (int l = 0; l + 1 < depth; l++)  // parents of level l push to level l + 1
        fmm::launch_l2l_level(g, p->level_begin[l], p->level_begin[l + 1], p->prm.p, level_parents(p, l),
                              p->ops_l2l.as<double>(), p->L.as<double>(), s);
    mark(p, ST_L2L);
    // L2P also writes the outputs (near + far, input order) when the near
    // field is complete; the far field stays for the energy and a later
    // fmm_backward
    fmm::FinalOut out;
    if (!deferred) {
        out.perm = p->idx.as<uint32_t>();
        out.qs = p->qs.as<double>();
        out.phi_near = p->phi_near.as<double>();
        out.fld_near = p->fld_near.as<double>();
        out.phi = phi;
        out.field = field;
        out.force = force;
    }
    fmm::launch_l2p(g, p->n, p->prm.p, p->leaf_of.as<int32_t>(), p->xs.as<double>(), p->ys.as<double>(),
                    p->zs.as<double>(), p->L.as<double>(), p->phi_far.as<double>(), p->fld_far.as<double>(), s, out);
    mark(p, ST_L2P);
    fmm::FinalOut out_e;   // outputs written by the energy pass (deferred queue with an energy)
    if (deferred) {
        fmm::near_far_tail(p->nf, a_nf, s);
        if (time_queue) {
            FMM_HIP_CHECK(hipEventRecord(p->ev_end[ST_QUEUE], fmm::near_far_join_stream(p->nf)));
            p->ev_used[ST_QUEUE] = true;
        }
        fmm::near_far_join(p->nf, s);
        join_guard.pending = false;
        if (energy && (phi || field || force)) {
            out_e.perm = p->idx.as<uint32_t>();
            out_e.qs = p->qs.as<double>();
            out_e.phi_near = p->phi_near.as<double>();
            out_e.fld_near = p->fld_near.as<double>();
            out_e.phi = phi;
            out_e.field = field;
            out_e.force = force;
        } else {
            fmm::launch_finalize(p->n, p->idx.as<uint32_t>(), p->qs.as<double>(), p->phi_near.as<double>(),
                                 p->fld_near.as<double>(), p->phi_far.as<double>(), p->fld_far.as<double>(), phi,
                                 field, force, s);
        }
    }
    if (energy)
        fmm::launch_energy(p->off.as<int64_t>(), p->n_inst, p->echunk.as<int32_t>(), p->nechunk, p->qs.as<double>(),
                           p->phi_near.as<double>(), p->phi_far.as<double>(),
                           p->epart_override ? p->epart_override : p->epart.as<double>(), energy, s, out_e,
                           p->fld_far.as<double>());
    mark(p, ST_OUT);
}

// Frozen-topology rebuild: new positions and charges through the stored
// permutation; box, keys, tree, lists and task tables stay.  check_leaf
// (incremental mode): also checks that every particle is still inside its
// leaf cell widened by 1/8 of its side; returns false if one is not (the
// caller then rebuilds).  Under graph capture nothing is read back: the
// flags stay on the device for fmm_sync.  With the P2P task durations the
// last evaluation on this topology measured (FMM_FLAG_COST_REUSE), the P2P
// tasks are reordered by them.
bool do_refresh(fmm_plan *p, const double *pos, const double *q, bool check_leaf) {
    hipStream_t s = p->stream;
    p->upward_fresh = false;   // new particles: fmm_upward recomputes
    int32_t *rflag = p->flag.as<int32_t>() + fmm::kRefreshFlag;   // the build's flags stay
    fmm::fill_zero(rflag, 2 * sizeof(int32_t), s);
    fmm::launch_gather(pos, q, p->idx.as<uint32_t>(), p->n, p->xs.as<double>(), p->ys.as<double>(), p->zs.as<double>(),
                       p->qs.as<double>(), s);
    fmm::launch_refresh_check(cells_of(p), p->leaf_of.as<int32_t>(), p->xs.as<double>(), p->ys.as<double>(),
                              p->zs.as<double>(), p->box.as<double>(), p->scale.as<double>(), p->n, check_leaf,
                              rflag, s);
    if (!p->capturing) {
        int32_t f[2] = {0, 0};
        sync_read(p, f, rflag, sizeof(f));
        if (f[0]) throw std::invalid_argument("non-finite particle coordinate");
        if (f[1]) return false;
    }
    if (cost_reuse(p) && p->leaf_cost_valid) {
        // device work only, so a captured step reorders at every replay by
        // the durations the previous replay measured
        fmm::NearFarArgs a = nf_args(p);
        a.leaf_cost = p->leaf_cost.as<float>();
        fmm::reorder_p2p_leaves(p->nf, a, s);
    }
    if (p->nf.built) start_near_early(p, s);
    return true;
}

fmm::NearFarArgs nf_args_adjoint(fmm_plan *p) {
    fmm::NearFarArgs a = nf_args(p);
    a.m2l_ptr = p->m2l_t_ptr.as<int32_t>();
    a.m2l_src = p->m2l_t_src.as<int32_t>();
    a.p2p_ptr = p->p2p_t_ptr.as<int32_t>();
    a.p2p_src = p->p2p_t_src.as<int32_t>();
    a.qs = p->wts.as<double>();
    a.M = p->lam.as<double>();
    a.L = p->mu.as<double>();
    a.phi = p->psi_near.as<double>();
    a.fld = p->epsi_near.as<double>();
    a.transposed = true;
    return a;
}

// Transposed M2L and P2P lists (and, mixed, the transposed queue tables).
void build_adjoint(fmm_plan *p) {
    hipStream_t s = p->stream;
    const int32_t ncell = (int32_t)p->ncell;
    const int bits = bits_for(ncell);
    const bool key32 = 2 * bits <= 32;
    const size_t ksz = key32 ? 4 : 8;
    const int64_t mx = std::max<int64_t>(std::max(p->nm2l, p->np2p), 1);
    FMM_HIP_CHECK(p->tkeys.grow(mx * ksz));
    FMM_HIP_CHECK(p->tkeys_alt.grow(mx * ksz));
    FMM_HIP_CHECK(p->tmp.grow(std::max(p->tmp.bytes, fmm::radix_tmp_elems(mx) * sizeof(int32_t))));
    FMM_HIP_CHECK(p->m2l_t_ptr.grow(((size_t)ncell + 1) * 4));
    FMM_HIP_CHECK(p->p2p_t_ptr.grow(((size_t)ncell + 1) * 4));
    FMM_HIP_CHECK(p->m2l_t_src.grow(std::max<int64_t>(p->nm2l, 1) * 4));
    FMM_HIP_CHECK(p->p2p_t_src.grow(std::max<int64_t>(p->np2p, 1) * 4));
    fmm::transpose_csr(p->m2l_ptr.as<int32_t>(), p->m2l_src.as<int32_t>(), ncell, p->nm2l, bits, key32, p->tkeys.ptr,
                       p->tkeys_alt.ptr, p->tmp.as<int32_t>(), p->m2l_t_ptr.as<int32_t>(), p->m2l_t_src.as<int32_t>(),
                       s);
    fmm::transpose_csr(p->p2p_ptr.as<int32_t>(), p->p2p_src.as<int32_t>(), ncell, p->np2p, bits, key32, p->tkeys.ptr,
                       p->tkeys_alt.ptr, p->tmp.as<int32_t>(), p->p2p_t_ptr.as<int32_t>(), p->p2p_t_src.as<int32_t>(),
                       s);
    if (p->prm.precision == FMM_PREC_MIXED || fmm::m2l_f64_supported(p->prm.p))
        fmm::build_near_far_mixed(p->nf_t, nf_args_adjoint(p), s);
    p->adj_ready = true;
}

void do_backward(fmm_plan *p, const double *gE, double *grad_pos, double *grad_q) {
    hipStream_t s = p->stream;
    const int pp = p->prm.p;
    const int P = fmm::ncoef(pp);
    const int32_t ncell = (int32_t)p->ncell;
    const size_t nn = (size_t)std::max<int64_t>(p->n, 1);
    ensure_ops(p);
    if (!p->adj_ready) build_adjoint(p);
    FMM_HIP_CHECK(p->lam.grow((size_t)std::max(ncell, 1) * P * 8));
    FMM_HIP_CHECK(p->mu.grow((size_t)std::max(ncell, 1) * P * 8));
    FMM_HIP_CHECK(p->wts.grow(nn * 8));
    FMM_HIP_CHECK(p->psi_near.grow(nn * 8));
    FMM_HIP_CHECK(p->epsi_near.grow(nn * 24));
    FMM_HIP_CHECK(p->psi_far.grow(nn * 8));
    FMM_HIP_CHECK(p->epsi_far.grow(nn * 24));
    fmm::Geometry g = geom(p);
    fmm::launch_adjoint_weights(g, p->n, p->leaf_of.as<int32_t>(), gE, p->qs.as<double>(), p->wts.as<double>(), s);
    // L2P^T at the leaves, then L2L^T up the tree
    fmm::launch_p2m(g, ncell, pp, p->xs.as<double>(), p->ys.as<double>(), p->zs.as<double>(), p->wts.as<double>(),
                    p->lam.as<double>(), s);
    fmm::launch_dual_scale(g, ncell, pp, p->lam.as<double>(), 0, s);
    const int depth = (int)p->level_begin.size() - 1;
    for (int l = depth - 2; l >= 0; l--)
        fmm::launch_m2m_level(g, p->level_begin[l], p->level_begin[l + 1], pp, level_parents(p, l),
                              p->ops_l2l_t.as<double>(), p->lam.as<double>(), p->m2m_part.as<double>(), s);
    // M2L^T and P2P^T
    if (p->prm.precision == FMM_PREC_FP64) {
        if (p->nf_t.built && p->nf_t.f64)
            fmm::m2l_f64_run(p->nf_t, nf_args_adjoint(p), s);
        else
            fmm::launch_m2l_fp64_adjoint(g, ncell, pp, p->m2l_t_ptr.as<int32_t>(), p->m2l_t_src.as<int32_t>(),
                                         p->nm2l, p->lam.as<double>(), p->mu.as<double>(), 0, deterministic(p), s);
        fmm::launch_p2p_fp64(g, ncell, p->p2p_t_ptr.as<int32_t>(), p->p2p_t_src.as<int32_t>(), p->xs.as<double>(),
                             p->ys.as<double>(), p->zs.as<double>(), p->wts.as<double>(), p->psi_near.as<double>(),
                             p->epsi_near.as<double>(), s);
    } else {
        fmm::NearFarArgs a = nf_args_adjoint(p);
        fmm::near_far_prepare(p->nf_t, a, s);
        fmm::near_far_queue(p->nf_t, a, s);
        fmm::near_far_rest(p->nf_t, a, s);
    }
    // M2M^T down the tree, then P2M^T at the particles
    for (int l = 0; l + 1 < depth; l++)
        fmm::launch_l2l_level(g, p->level_begin[l], p->level_begin[l + 1], pp, level_parents(p, l),
                              p->ops_m2m_t.as<double>(), p->mu.as<double>(), s);
    fmm::launch_dual_scale(g, ncell, pp, p->mu.as<double>(), 1, s);
    fmm::launch_l2p(g, p->n, pp, p->leaf_of.as<int32_t>(), p->xs.as<double>(), p->ys.as<double>(), p->zs.as<double>(),
                    p->mu.as<double>(), p->psi_far.as<double>(), p->epsi_far.as<double>(), s);
    fmm::launch_adjoint_finalize(g, p->n, p->idx.as<uint32_t>(), p->leaf_of.as<int32_t>(), gE, p->qs.as<double>(),
                                 p->phi_near.as<double>(), p->fld_near.as<double>(), p->phi_far.as<double>(),
                                 p->fld_far.as<double>(), p->psi_near.as<double>(), p->epsi_near.as<double>(),
                                 p->psi_far.as<double>(), p->epsi_far.as<double>(), grad_pos, grad_q, s);
}

template <class F>
fmm_status guarded(fmm_plan *p, F &&f) {
    try {
        if (p) {
            hipError_t e = hipSetDevice(p->device);
            if (e != hipSuccess) return fail(p, FMM_ERR_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
        }
        return f();
    } catch (const fmm::HipError &e) {
        if (e.err == hipErrorOutOfMemory) return fail(p, FMM_ERR_OOM, std::string("out of device memory: ") + e.what);
        return fail(p, FMM_ERR_DEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
    } catch (const std::invalid_argument &e) {
        return fail(p, FMM_ERR_INVALID_ARG, e.what());
    } catch (const fmm::NoAllocError &e) {
        return fail(p, FMM_ERR_STATE, std::string(e.what()) + " (call fmm_evaluate once to size the workspaces)");
    } catch (const std::bad_alloc &) {
        return fail(p, FMM_ERR_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(p, FMM_ERR_DEVICE, e.what());
    }
}

fmm_status check_params(const fmm_params *q, std::string *why) {
    if (q->p < 0 || q->p > fmm::kMaxP) return *why = "p must be in [0, 16]", FMM_ERR_INVALID_ARG;
    if (q->ncrit < 1) return *why = "ncrit must be >= 1", FMM_ERR_INVALID_ARG;
    if (q->theta_num < 1 || q->theta_den < 1 || q->theta_num > 100 || q->theta_den > 100 ||
        q->theta_num >= q->theta_den)
        return *why = "theta must be num/den with 1 <= num < den <= 100", FMM_ERR_INVALID_ARG;
    if ((q->flags & FMM_FLAG_INCREMENTAL) && 5 * q->theta_num >= 4 * q->theta_den)
        return *why = "FMM_FLAG_INCREMENTAL needs theta < 4/5 (cells widened by 1/8 of a side)", FMM_ERR_INVALID_ARG;
    if (q->max_level < 1 || q->max_level > fmm::kLevels) return *why = "max_level must be in [1, 21]", FMM_ERR_INVALID_ARG;
    if (q->precision != FMM_PREC_FP64 && q->precision != FMM_PREC_MIXED)
        return *why = "unknown precision", FMM_ERR_INVALID_ARG;
    if (q->flags & ~(uint32_t)(FMM_FLAG_USER_BOX | FMM_FLAG_KEEP_TOPOLOGY | FMM_FLAG_TRACE | FMM_FLAG_DETERMINISTIC |
                               FMM_FLAG_INCREMENTAL | FMM_FLAG_COST_REUSE | FMM_FLAG_MUTUAL_M2L |
                               FMM_FLAG_MUTUAL_P2P))
        return *why = "unknown flag", FMM_ERR_INVALID_ARG;
    if ((q->flags & FMM_FLAG_MUTUAL) && q->precision != FMM_PREC_FP64)
        return *why = "the mutual flags need FMM_PREC_FP64", FMM_ERR_INVALID_ARG;
    if ((q->flags & FMM_FLAG_MUTUAL) && (q->flags & FMM_FLAG_DETERMINISTIC))
        return *why = "the mutual flags add with atomics: not with FMM_FLAG_DETERMINISTIC", FMM_ERR_INVALID_ARG;
    if ((q->flags & FMM_FLAG_USER_BOX) &&
        !(q->box_side > 0 && std::isfinite(q->box_side) && std::isfinite(q->box_min[0]) &&
          std::isfinite(q->box_min[1]) && std::isfinite(q->box_min[2])))
        return *why = "user box must be finite with side > 0", FMM_ERR_INVALID_ARG;
    return FMM_OK;
}

}  // namespace

extern "C" {

fmm_status fmm_default_params(fmm_params *params) {
    if (!params) return FMM_ERR_INVALID_ARG;
    std::memset(params, 0, sizeof(*params));
    params->p = 8;
    params->ncrit = 64;
    params->theta_num = 1;
    params->theta_den = 2;
    params->max_level = fmm::kLevels;
    params->precision = FMM_PREC_MIXED;
    params->flags = 0;
    params->box_side = 1.0;
    return FMM_OK;
}

fmm_status fmm_create(const fmm_params *params, int device, void *hip_stream, fmm_plan **out) {
    if (!params || !out) return FMM_ERR_INVALID_ARG;
    *out = nullptr;
    std::string why;
    fmm_status st = check_params(params, &why);
    if (st != FMM_OK) return st;
    if (device < 0) return FMM_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return FMM_ERR_DEVICE;
    fmm_plan *p = new (std::nothrow) fmm_plan();
    if (!p) return FMM_ERR_OOM;
    p->prm = *params;
    p->device = device;
    p->stream = (hipStream_t)hip_stream;
    p->tuning = fmm::default_tuning();
    // the FP64 matrix-core M2L runs its tasks as one plain launch (no queue
    // to balance them): smaller tasks fill the chip more evenly
    if (params->precision == FMM_PREC_FP64) p->tuning.m2l_task_entries = fmm::kFp64TaskEntries;
    if (hipSetDevice(device) != hipSuccess) {
        delete p;
        return FMM_ERR_DEVICE;
    }
    p->reader.init();
    (void)fmm::scratch_on(device);   // resolved once per device, before any no-allocation call
    p->ev_ok = true;
    for (int i = 0; i < ST_COUNT; i++)
        if (hipEventCreate(&p->ev_beg[i]) != hipSuccess || hipEventCreate(&p->ev_end[i]) != hipSuccess)
            p->ev_ok = false;
    if (hipEventCreate(&p->ev_early) != hipSuccess) p->ev_ok = false;
    *out = p;
    return FMM_OK;
}

fmm_status fmm_destroy(fmm_plan *p) {
    if (!p) return FMM_OK;
    hipSetDevice(p->device);
    // every stream that may still run kernels on plan memory drains before
    // any buffer is released: the plan's stream, the build's second stream
    // (an interrupted build) and the side streams of both work queues (a
    // P2P tail whose join was never enqueued)
    hipStreamSynchronize(p->stream);
    hipStream_t others[] = {p->up_side, p->nf.side, p->nf.side2, p->nf_t.side, p->nf_t.side2};
    for (hipStream_t o : others)
        if (o) hipStreamSynchronize(o);
    DevBuf *all[] = {&p->off, &p->ord, &p->flag, &p->box, &p->scale, &p->keys, &p->kalt, &p->idx, &p->valt,
                     &p->ikey, &p->ialt, &p->rank, &p->ralt, &p->tmp, &p->xs, &p->ys, &p->zs, &p->qs,
                     &p->leaf_of, &p->bounds, &p->nch, &p->counters, &p->front[0], &p->front[1], &p->m2l_pairs,
                     &p->p2p_pairs, &p->pair_alt, &p->m2l_ptr, &p->m2l_src, &p->p2p_ptr, &p->p2p_src, &p->M,
                     &p->L, &p->ops_m2m, &p->ops_l2l, &p->m2m_part, &p->phi_near, &p->fld_near, &p->phi_far,
                     &p->fld_far, &p->echunk, &p->epart, &p->ops_m2m_t, &p->ops_l2l_t, &p->m2l_t_ptr,
                     &p->m2l_t_src, &p->p2p_t_ptr, &p->p2p_t_src, &p->tkeys, &p->tkeys_alt, &p->lam, &p->mu,
                     &p->wts, &p->psi_near, &p->epsi_near, &p->psi_far, &p->epsi_far, &p->trace,
                     &p->trace_count, &p->pair_alt2, &p->tmp2, &p->leaf_cost, &p->ppos, &p->plist, &p->ptmp};
    drop_graph(p);
    for (DevBuf *b : all) b->release();
    for (auto &b : p->cb) b.release();
    p->crec.release();
    p->levdev.release();
    if (p->up_side) {
        (void)hipStreamDestroy(p->up_side);
        (void)hipEventDestroy(p->up_fork);
        (void)hipEventDestroy(p->up_join);
        (void)hipEventDestroy(p->p2p_fork);
        (void)hipEventDestroy(p->p2p_done);
    }
    fmm::release_near_far(p->nf);
    fmm::release_near_far(p->nf_t);
    p->reader.release();
    for (int i = 0; i < ST_COUNT; i++) {
        if (p->ev_beg[i]) hipEventDestroy(p->ev_beg[i]);
        if (p->ev_end[i]) hipEventDestroy(p->ev_end[i]);
    }
    if (p->ev_early) hipEventDestroy(p->ev_early);
    delete p;
    return FMM_OK;
}

fmm_status fmm_build_tree(fmm_plan *p, int32_t n_inst, const int64_t *offsets, const double *pos, const double *q) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (n_inst < 1 || !offsets) return fail(p, FMM_ERR_INVALID_ARG, "n_inst >= 1 and offsets required");
    if (offsets[0] != 0) return fail(p, FMM_ERR_INVALID_ARG, "offsets[0] must be 0");
    for (int k = 0; k < n_inst; k++)
        if (offsets[k + 1] < offsets[k]) return fail(p, FMM_ERR_INVALID_ARG, "offsets must be non-decreasing");
    int64_t n = offsets[n_inst];
    if (n >= ((int64_t)1 << 31) - 1) return fail(p, FMM_ERR_INVALID_ARG, "too many particles (limit 2^31 - 2)");
    if (n > 0 && (!pos || !q)) return fail(p, FMM_ERR_INVALID_ARG, "pos and q required");
    const bool same = p->state >= kStateBuilt && n_inst == p->n_inst &&
                      std::equal(offsets, offsets + n_inst + 1, p->h_off.begin());
    const bool keep = same && (p->prm.flags & FMM_FLAG_KEEP_TOPOLOGY);
    const bool incremental = same && !keep && (p->prm.flags & FMM_FLAG_INCREMENTAL);
    return guarded(p, [&]() -> fmm_status {
        // a near field started for the previous particles and never joined
        // must end before its inputs change
        fmm::near_far_drop_early(p->nf, p->stream);
        if ((keep || incremental) && n > 0) {
            const int saved = p->state;
            p->state = kStateBuilt;
            if (do_refresh(p, pos, q, incremental)) {
                p->nbuild_kept++;
                return FMM_OK;
            }
            p->state = saved;   // a particle left its leaf: rebuild from these positions
        }
        p->state = kStateCreated;
        p->adj_ready = false;
        p->traced = false;
        p->leaf_cost_valid = false;
        p->nbuild_full++;
        drop_graph(p);
        p->n = n;
        p->n_inst = n_inst;
        p->h_off.assign(offsets, offsets + n_inst + 1);
        for (bool &u : p->ev_used) u = false;
        p->last_ev = nullptr;
        do_build(p, pos, q);
        if (cost_reuse(p)) FMM_HIP_CHECK(p->leaf_cost.grow((size_t)std::max<int64_t>(p->ncell, 1) * sizeof(float)));
        p->state = kStateBuilt;
        return FMM_OK;
    });
}

fmm_status fmm_upward(fmm_plan *p) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return fail(p, FMM_ERR_STATE, "fmm_upward before fmm_build_tree");
    return guarded(p, [&]() -> fmm_status {
        do_upward(p);
        p->state = kStateUp;
        return FMM_OK;
    });
}

fmm_status fmm_evaluate(fmm_plan *p, double *phi, double *field, double *force, double *energy) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateUp) return fail(p, FMM_ERR_STATE, "fmm_evaluate before fmm_upward");
    return guarded(p, [&]() -> fmm_status {
        do_evaluate(p, phi, field, force, energy);
        p->state = kStateEval;
        return FMM_OK;
    });
}

fmm_status fmm_evaluate_noalloc(fmm_plan *p, double *phi, double *field, double *force, double *energy) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateUp) return fail(p, FMM_ERR_STATE, "fmm_evaluate_noalloc before fmm_upward");
    if (energy && p->nechunk > fmm::kScratchMaxChunks)
        return fail(p, FMM_ERR_CAPACITY,
                    "fmm_evaluate_noalloc: the energy needs " + std::to_string(p->nechunk) +
                        " chunk partials, more than the scratch array holds (" +
                        std::to_string(fmm::kScratchMaxChunks) + ")");
    if (p->prm.precision == FMM_PREC_MIXED && p->tuning.p2p_per_cu > 0 && !p->nf.side)
        return fail(p, FMM_ERR_STATE, "fmm_evaluate_noalloc: the work queue's side streams do not exist yet "
                                      "(call fmm_evaluate once)");
    return guarded(p, [&]() -> fmm_status {
        unsigned char *base = static_cast<unsigned char *>(fmm::scratch_on(p->device));
        if (!base) return fail(p, FMM_ERR_DEVICE, "fmm_evaluate_noalloc: the scratch array has no device address");
        // every workspace the evaluation grows must be large enough already
        struct Scope {
            fmm_plan *p;
            ~Scope() {
                fmm::t_no_alloc = false;
                p->heads_override = nullptr;
                p->epart_override = nullptr;
            }
        } scope{p};
        fmm::t_no_alloc = true;
        p->heads_override = reinterpret_cast<int32_t *>(base);
        p->epart_override = reinterpret_cast<double *>(base + fmm::kScratchHeads);
        do_evaluate(p, phi, field, force, energy);
        p->state = kStateEval;
        return FMM_OK;
    });
}

fmm_status fmm_backward(fmm_plan *p, const double *grad_energy, double *grad_pos, double *grad_q) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateEval) return fail(p, FMM_ERR_STATE, "fmm_backward before fmm_evaluate");
    if (!grad_energy) return fail(p, FMM_ERR_INVALID_ARG, "grad_energy required");
    if (p->n == 0) return FMM_OK;
    return guarded(p, [&]() -> fmm_status {
        do_backward(p, grad_energy, grad_pos, grad_q);
        return FMM_OK;
    });
}

namespace {
// Record a solve into the plan's graph: run it once eagerly (sizing every
// workspace), synchronise, then capture the same calls on a private stream
// (the plan's stream may be the legacy null stream, which cannot be
// captured) and instantiate.  step_pos / step_q: the solve starts with a
// frozen-topology rebuild from them.
void capture_solve(fmm_plan *p, const double *step_pos, const double *step_q, double *phi, double *field, double *force,
                   double *energy, const double *grad_energy, double *grad_pos, double *grad_q) {
    drop_graph(p);
    const bool check_leaf = (p->prm.flags & FMM_FLAG_INCREMENTAL) != 0;
    auto solve = [&]() {
        if (step_pos) {
            if (!do_refresh(p, step_pos, step_q, check_leaf))
                throw std::invalid_argument("a particle is outside its leaf cell: rebuild the tree before capturing");
            if (!p->capturing) p->nbuild_kept++;
        }
        do_upward(p);
        do_evaluate(p, phi, field, force, energy);
        if (grad_energy) do_backward(p, grad_energy, grad_pos, grad_q);
    };
    solve();
    p->state = kStateEval;
    FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
    hipStream_t cs = nullptr;
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));   // default priority
    hipStream_t saved = p->stream;
    p->stream = cs;
    p->capturing = true;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    hipGraph_t g = nullptr;
    if (e == hipSuccess) {
        try {
            solve();
        } catch (...) {
            hipStreamEndCapture(cs, &g);
            if (g) hipGraphDestroy(g);
            p->capturing = false;
            p->stream = saved;
            hipStreamDestroy(cs);
            throw;
        }
        e = hipStreamEndCapture(cs, &g);
    }
    p->capturing = false;
    p->stream = saved;
    hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        throw fmm::HipError{e, "stream capture"};
    }
    p->graph = g;
    FMM_HIP_CHECK(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
    p->graph_step = step_pos != nullptr;
}
}  // namespace

fmm_status fmm_graph_capture(fmm_plan *p, double *phi, double *field, double *force, double *energy,
                             const double *grad_energy, double *grad_pos, double *grad_q) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return fail(p, FMM_ERR_STATE, "fmm_graph_capture before fmm_build_tree");
    if (p->n == 0) return fail(p, FMM_ERR_INVALID_ARG, "nothing to capture (N = 0)");
    return guarded(p, [&]() -> fmm_status {
        capture_solve(p, nullptr, nullptr, phi, field, force, energy, grad_energy, grad_pos, grad_q);
        return FMM_OK;
    });
}

fmm_status fmm_graph_capture_step(fmm_plan *p, const double *pos, const double *q, double *phi, double *field,
                                  double *force, double *energy) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return fail(p, FMM_ERR_STATE, "fmm_graph_capture_step before fmm_build_tree");
    if (!(p->prm.flags & (FMM_FLAG_KEEP_TOPOLOGY | FMM_FLAG_INCREMENTAL)))
        return fail(p, FMM_ERR_STATE, "fmm_graph_capture_step needs FMM_FLAG_KEEP_TOPOLOGY or FMM_FLAG_INCREMENTAL");
    if (p->n == 0) return fail(p, FMM_ERR_INVALID_ARG, "nothing to capture (N = 0)");
    if (!pos || !q) return fail(p, FMM_ERR_INVALID_ARG, "pos and q required");
    return guarded(p, [&]() -> fmm_status {
        capture_solve(p, pos, q, phi, field, force, energy, nullptr, nullptr, nullptr);
        return FMM_OK;
    });
}

fmm_status fmm_get_build_info(const fmm_plan *p, int64_t *full_builds, int64_t *kept_builds) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (full_builds) *full_builds = p->nbuild_full;
    if (kept_builds) *kept_builds = p->nbuild_kept;
    return FMM_OK;
}

fmm_status fmm_graph_launch(fmm_plan *p) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (!p->graph_exec) return fail(p, FMM_ERR_STATE, "fmm_graph_launch without a captured graph");
    if (p->state < kStateBuilt) return fail(p, FMM_ERR_STATE, "fmm_graph_launch after the tree was dropped");
    return guarded(p, [&]() -> fmm_status {
        FMM_HIP_CHECK(hipGraphLaunch(p->graph_exec, p->stream));
        p->state = kStateEval;
        return FMM_OK;
    });
}

fmm_status fmm_sync(fmm_plan *p) {
    if (!p) return FMM_ERR_INVALID_ARG;
    return guarded(p, [&]() -> fmm_status {
        FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
        if (p->graph_step && p->flag.ptr) {   // the checks of a replayed frozen-topology rebuild
            int32_t f[2] = {0, 0};
            FMM_HIP_CHECK(hipMemcpy(f, p->flag.as<int32_t>() + fmm::kRefreshFlag, sizeof(f), hipMemcpyDeviceToHost));
            if (f[0]) return fail(p, FMM_ERR_INVALID_ARG, "non-finite particle coordinate in the replayed step");
            if (f[1])
                return fail(p, FMM_ERR_STATE, "a particle left its leaf cell in the replayed step: rebuild the tree");
        }
        return FMM_OK;
    });
}

fmm_status fmm_get_counts(const fmm_plan *p, int64_t *ncell, int64_t *nleaf, int64_t *nm2l, int64_t *np2p) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return FMM_ERR_STATE;
    if (ncell) *ncell = p->ncell;
    if (nleaf) *nleaf = p->nleaf;
    if (nm2l) *nm2l = p->nm2l;
    if (np2p) *np2p = p->np2p;
    return FMM_OK;
}

fmm_status fmm_get_queue_info(const fmm_plan *p, int64_t *ntarget, int64_t *ngroup, int64_t *ntask, int64_t *nclass,
                              int64_t *nextra) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return FMM_ERR_STATE;
    const bool q = p->nf.built;
    if (ntarget) *ntarget = q ? p->nf.ntarget : 0;
    if (ngroup) *ngroup = q ? p->nf.ngroup : 0;
    if (ntask) *ntask = q ? p->nf.ntask : 0;
    if (nclass) *nclass = q ? p->nf.nslot : 0;
    if (nextra) *nextra = q ? p->nf.nextra : 0;
    return FMM_OK;
}

fmm_status fmm_copy_tree(const fmm_plan *cp, uint64_t *keys, int64_t *perm, int64_t *cells) {
    fmm_plan *p = const_cast<fmm_plan *>(cp);
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return fail(p, FMM_ERR_STATE, "no tree");
    return guarded(p, [&]() -> fmm_status {
        const int64_t n = p->n;
        if (n > 0 && (keys || perm)) {
            std::vector<uint64_t> sk(n);
            std::vector<uint32_t> ix(n);
            FMM_HIP_CHECK(hipMemcpyAsync(sk.data(), p->keys.ptr, n * 8, hipMemcpyDeviceToHost, p->stream));
            FMM_HIP_CHECK(hipMemcpyAsync(ix.data(), p->idx.ptr, n * 4, hipMemcpyDeviceToHost, p->stream));
            FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
            for (int64_t r = 0; r < n; r++) {
                if (keys) keys[ix[r]] = sk[r];
                if (perm) perm[r] = ix[r];
            }
        }
        if (cells && p->ncell > 0) {
            std::vector<int32_t> col(p->ncell);
            for (int f = 0; f < 10; f++) {
                FMM_HIP_CHECK(hipMemcpyAsync(col.data(), p->cb[f].ptr, p->ncell * 4, hipMemcpyDeviceToHost, p->stream));
                FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
                for (int64_t c = 0; c < p->ncell; c++) cells[c * 10 + f] = col[c];
            }
        }
        return FMM_OK;
    });
}

fmm_status fmm_copy_lists(const fmm_plan *cp, int64_t *m2l_ptr, int32_t *m2l_src, int64_t *p2p_ptr, int32_t *p2p_src) {
    fmm_plan *p = const_cast<fmm_plan *>(cp);
    if (!p) return FMM_ERR_INVALID_ARG;
    if (p->state < kStateBuilt) return fail(p, FMM_ERR_STATE, "no lists");
    return guarded(p, [&]() -> fmm_status {
        const int64_t nc1 = p->ncell + 1;
        std::vector<int32_t> tmp(nc1);
        int64_t *outs[2] = {m2l_ptr, p2p_ptr};
        int32_t *srcs[2] = {m2l_src, p2p_src};
        DevBuf *ptrs[2] = {&p->m2l_ptr, &p->p2p_ptr};
        DevBuf *dsrc[2] = {&p->m2l_src, &p->p2p_src};
        const int64_t cnts[2] = {p->nm2l, p->np2p};
        for (int t = 0; t < 2; t++) {
            if (!outs[t] && !srcs[t]) continue;
            FMM_HIP_CHECK(hipMemcpyAsync(tmp.data(), ptrs[t]->ptr, nc1 * 4, hipMemcpyDeviceToHost, p->stream));
            if (srcs[t] && cnts[t] > 0)
                FMM_HIP_CHECK(hipMemcpyAsync(srcs[t], dsrc[t]->ptr, cnts[t] * 4, hipMemcpyDeviceToHost, p->stream));
            FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
            if (outs[t])
                for (int64_t i = 0; i < nc1; i++) outs[t][i] = tmp[i];
            if (srcs[t])   // canonical order: each target's sources ascending
                for (int64_t i = 0; i + 1 < nc1; i++) std::sort(srcs[t] + tmp[i], srcs[t] + tmp[i + 1]);
        }
        return FMM_OK;
    });
}

fmm_status fmm_get_tuning(const fmm_plan *p, fmm_tuning *t) {
    if (!p || !t) return FMM_ERR_INVALID_ARG;
    *t = p->tuning;
    return FMM_OK;
}

fmm_status fmm_set_tuning(fmm_plan *p, const fmm_tuning *t) {
    if (!p || !t) return FMM_ERR_INVALID_ARG;
    if (t->m2l_task_entries < 1 || t->m2l_task_entries > 128 || t->grid_per_cu < 1 || t->grid_per_cu > 8 ||
        t->p2p_per_cu < 0 || t->p2p_per_cu > 8 || t->early_p2p_per_cu < 0 || t->early_p2p_per_cu > t->p2p_per_cu)
        return fail(p, FMM_ERR_INVALID_ARG, "tuning out of range");
    p->tuning = *t;
    return FMM_OK;
}

fmm_status fmm_autotune(fmm_plan *p, int32_t repeats, fmm_tuning *best, double *best_ms) {
    if (!p) return FMM_ERR_INVALID_ARG;
    if (repeats < 1) return fail(p, FMM_ERR_INVALID_ARG, "repeats must be >= 1");
    if (p->state < kStateUp) return fail(p, FMM_ERR_STATE, "fmm_autotune before fmm_upward");
    // the FP64 path tunes the task size of its matrix-core M2L (over the
    // class tables; nothing to tune where M2L runs per pair)
    const bool fp64 = p->prm.precision == FMM_PREC_FP64;
    if (p->n == 0 || (fp64 && !(p->nf.built && p->nf.f64))) {
        if (best) *best = p->tuning;
        if (best_ms) *best_ms = -1.0;
        return FMM_OK;
    }
    return guarded(p, [&]() -> fmm_status {
        hipStream_t s = p->stream;
        drop_graph(p);
        p->adj_ready = false;
        fmm::near_far_drop_early(p->nf, s);   // every trial launches its own near field
        ensure_eval_buffers(p);   // the queue writes the locals and the near field
        static const int kEntries[] = {32, 64, 96, 128};
        static const int kEntries64[] = {16, 32, 64, 128};
        // (work-queue, P2P side) workgroups per compute unit; the early near
        // field stays as set (its gain depends on what the build lets it
        // overlap, which one evaluation does not show)
        static const int kShape[][3] = {{1, 1, 0}, {1, 2, 0}, {1, 3, 0}, {2, 0, 0}, {3, 0, 0}, {2, 1, 0}, {2, 2, 0}};
        const int nshape = fp64 ? 1 : (int)(sizeof(kShape) / sizeof(kShape[0]));   // FP64: no queue to shape
        hipEvent_t e0, e1;
        FMM_HIP_CHECK(hipEventCreate(&e0));
        FMM_HIP_CHECK(hipEventCreate(&e1));
        fmm_tuning keep = p->tuning, top = keep;
        float top_ms = -1.0f;
        try {
            for (int ei = 0; ei < 4; ei++) {
                p->tuning.m2l_task_entries = fp64 ? kEntries64[ei] : kEntries[ei];
                fmm::build_near_far_mixed(p->nf, nf_args(p), s);
                for (int si = 0; si < nshape; si++) {
                    if (!fp64) {
                        const int *sh = kShape[si];
                        p->tuning.grid_per_cu = sh[0];
                        p->tuning.p2p_per_cu = sh[1];
                        p->tuning.early_p2p_per_cu = std::min(keep.early_p2p_per_cu, sh[1]);
                    }
                    float t_min = -1.0f;
                    for (int r = 0; r < repeats; r++) {
                        // the whole evaluation (queue, far field beside the
                        // P2P tail, join), no outputs
                        FMM_HIP_CHECK(hipEventRecord(e0, s));
                        do_evaluate(p, nullptr, nullptr, nullptr, nullptr);
                        FMM_HIP_CHECK(hipEventRecord(e1, s));
                        FMM_HIP_CHECK(hipEventSynchronize(e1));
                        float ms = 0.0f;
                        FMM_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                        if (t_min < 0.0f || ms < t_min) t_min = ms;
                    }
                    if (top_ms < 0.0f || t_min < top_ms) {
                        top_ms = t_min;
                        top = p->tuning;
                    }
                }
            }
            p->tuning = top;
            fmm::build_near_far_mixed(p->nf, nf_args(p), s);
        } catch (...) {
            p->tuning = keep;
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            throw;
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        p->state = kStateUp;
        if (best) *best = top;
        if (best_ms) *best_ms = top_ms;
        return FMM_OK;
    });
}

fmm_status fmm_get_trace(const fmm_plan *cp, fmm_task_record *records, int64_t cap, int64_t *count) {
    fmm_plan *p = const_cast<fmm_plan *>(cp);
    if (!p || cap < 0 || (cap > 0 && !records)) return FMM_ERR_INVALID_ARG;
    return guarded(p, [&]() -> fmm_status {
        int32_t n = 0;
        if (p->traced && p->trace_count.ptr) {
            FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
            FMM_HIP_CHECK(hipMemcpy(&n, p->trace_count.ptr, sizeof(int32_t), hipMemcpyDeviceToHost));
            n = std::min(n, p->trace_cap);
        }
        if (count) *count = n;
        const int64_t m = std::min<int64_t>(n, cap);
        if (m > 0)
            FMM_HIP_CHECK(hipMemcpy(records, p->trace.ptr, (size_t)m * sizeof(fmm_task_record), hipMemcpyDeviceToHost));
        return FMM_OK;
    });
}

fmm_status fmm_get_stage_times(const fmm_plan *cp, double *times, const char **names) {
    fmm_plan *p = const_cast<fmm_plan *>(cp);
    if (!p || !times) return FMM_ERR_INVALID_ARG;
    return guarded(p, [&]() -> fmm_status {
        FMM_HIP_CHECK(hipStreamSynchronize(p->stream));
        for (int i = 0; i < 16; i++) {
            times[i] = 0.0;
            if (names) names[i] = kStageNames[i];
        }
        if (!p->ev_ok) return FMM_OK;
        for (int i = 0; i < ST_COUNT; i++) {
            if (!p->ev_used[i]) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p->beg_of[i], p->ev_end[i]) == hipSuccess) times[i] = ms;
        }
        return FMM_OK;
    });
}

const char *fmm_status_string(fmm_status s) {
    switch (s) {
        case FMM_OK: return "ok";
        case FMM_ERR_INVALID_ARG: return "invalid argument";
        case FMM_ERR_STATE: return "call out of order";
        case FMM_ERR_OOM: return "out of memory";
        case FMM_ERR_DEVICE: return "device error";
        case FMM_ERR_CAPACITY: return "capacity exceeded";
        case FMM_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *fmm_last_error(const fmm_plan *p) {
    if (!p) return "null plan";
    return p->err.c_str();
}

}  // extern "C"
