// Orchestration of the mixed-precision near/far field stage.
#include <algorithm>
#include <stdexcept>

#include "m2l_mfma.h"
#include "near_far.h"
#include "queue.h"

namespace fmm {

fmm_tuning default_tuning() {
    fmm_tuning t;
    t.m2l_task_entries = 128;
    t.grid_per_cu = 1;
    t.p2p_per_cu = 2;
    t.early_p2p_per_cu = 0;
    return t;
}

namespace {
// Device-to-host reads in two halves (see HostReader): work enqueued
// between read_begin and read_end runs while the host waits.
struct Reader {
    const NearFarArgs &a;
    const void *d = nullptr;
    size_t b = 0;
    void begin(const void *dev, size_t bytes, hipStream_t s) {
        d = dev;
        b = bytes;
        if (a.reader) a.reader->begin(dev, bytes, s);
    }
    void end(void *host, hipStream_t s) {
        if (a.reader) {
            a.reader->end(host, s);
        } else {
            FMM_HIP_CHECK(hipMemcpyAsync(host, d, b, hipMemcpyDeviceToHost, s));
            FMM_HIP_CHECK(hipStreamSynchronize(s));
        }
    }
};

// The 16 task lists from the per-XCD counts: list 2x = (first task,
// count, 0, 0) from the M2L task counts hc[0..7] (kind 0); list 2x + 1 =
// (0, leaves, first leaf, 0) from the leaf counts hc[0..7] (kind 1).  The
// two halves are written by different streams and never overlap.
__global__ void k_make_lists(const int32_t *__restrict__ hc, int kind, int4 *__restrict__ lists) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t first = 0;
    for (int x = 0; x < 8; x++) {
        lists[2 * x + kind] = kind == 0 ? make_int4(first, hc[x], 0, 0) : make_int4(0, hc[x], first, 0);
        first += hc[x];
    }
}
}  // namespace

void build_near_far_mixed(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    const int p = a.p;
    if (a.f64 ? !m2l_f64_supported(p) : !queue_supported(p))
        throw std::runtime_error("the class-batched M2L supports p <= 12");
    const int RT = queue_row_tiles(p);
    const int64_t op_elems = queue_op_elems(p);
    const int32_t ncell = a.ncell;
    const int64_t npair = a.nm2l;
    // ---- persistent class tables (slot_of, the operator store, and the
    // key marks, which the slot allocation clears after each build).  The
    // order of a group's entries follows the operator slots, and the slots
    // follow the order in which classes are first seen; in deterministic
    // mode the store is therefore emptied at every build and refilled in
    // key order, so the entries (and the FP32 sums of each task) come in
    // the same order whatever the plan saw before.
    if (st.p != p || a.deterministic) {
        FMM_HIP_CHECK(st.slot_of.grow(kDenseKeys * 4));
        FMM_HIP_CHECK(hipMemsetAsync(st.slot_of.ptr, 0xff, kDenseKeys * 4, s));
        FMM_HIP_CHECK(st.nslots.grow(2 * 4));
        FMM_HIP_CHECK(hipMemsetAsync(st.nslots.ptr, 0, 2 * 4, s));
        FMM_HIP_CHECK(st.used.grow(kDenseKeys * 4));
        FMM_HIP_CHECK(hipMemsetAsync(st.used.ptr, 0, kDenseKeys * 4, s));
        st.nslot_total = 0;
        st.p = p;
    }
    FMM_HIP_CHECK(st.new_keys.grow(kDenseKeys * 4));
    const size_t np1 = (size_t)std::max<int64_t>(npair, 1) + 1;
    FMM_HIP_CHECK(st.pcode.grow(np1 * 4));
    FMM_HIP_CHECK(st.xcount.grow(((size_t)ncell + 1) * 4));   // per-owner counts of pairs outside the table
    FMM_HIP_CHECK(st.xptr.grow(((size_t)ncell + 1) * 4));
    FMM_HIP_CHECK(st.cnt.grow(64 * 4));  // [0..4] sizes, [16..32] per-XCD counts, [40..55] queue heads
    int64_t tmp_elems = std::max<int64_t>({(int64_t)scan_tmp_elems(np1), (int64_t)radix_tmp_elems(ncell + 1),
                                           (int64_t)scan_tmp_elems(ncell + 1), (int64_t)scan_tmp_elems(kDenseKeys)});
    FMM_HIP_CHECK(st.tmp.grow(tmp_elems * 4));
    int32_t *cnt = st.cnt.as<int32_t>();

    m2l_pair_codes(a.g.c, ncell, a.m2l_ptr, a.m2l_src, st.slot_of.as<int32_t>(), st.pcode.as<int32_t>(),
                   st.used.as<int32_t>(), st.xcount.as<int32_t>(), s);
    FMM_HIP_CHECK(hipMemsetAsync(st.nslots.as<int32_t>() + 1, 0, 4, s));
    if (a.deterministic) {
        FMM_HIP_CHECK(st.key_rank.grow(((size_t)kDenseKeys + 1) * 4));
        m2l_alloc_slots_ordered(st.used.as<int32_t>(), st.slot_of.as<int32_t>(), st.nslots.as<int32_t>(),
                                st.new_keys.as<int32_t>(), st.key_rank.as<int32_t>(), st.tmp.as<int32_t>(), s);
    } else {
        m2l_alloc_slots(st.used.as<int32_t>(), st.slot_of.as<int32_t>(), st.nslots.as<int32_t>(),
                        st.new_keys.as<int32_t>(), s);
    }
    // slot counts next to the sizes below: one read for all of them
    FMM_HIP_CHECK(hipMemcpyAsync(cnt + 5, st.nslots.ptr, 8, hipMemcpyDeviceToDevice, s));
    // CSR offsets of the pairs left to the per-pair kernel; xptr[ncell] (and
    // cnt[1]) = their number
    exclusive_scan_oop(st.xcount.as<int32_t>(), st.xptr.as<int32_t>(), ncell, st.xptr.as<int32_t>() + ncell,
                       st.tmp.as<int32_t>(), s);
    FMM_HIP_CHECK(hipMemcpyAsync(cnt + 1, st.xptr.as<int32_t>() + ncell, 4, hipMemcpyDeviceToDevice, s));
    // ---- targets sorted by (level, octant, cell)
    FMM_HIP_CHECK(st.tkey.grow((size_t)(ncell + 1) * 8));
    FMM_HIP_CHECK(st.tkey_alt.grow((size_t)(ncell + 1) * 8));
    FMM_HIP_CHECK(st.has.grow((size_t)(ncell + 1) * 4));
    m2l_target_keys(a.g.c, ncell, a.n, a.m2l_ptr, st.xptr.as<int32_t>(), st.tkey.as<uint64_t>(), st.has.as<int32_t>(),
                    s);
    // the keys are written in cell order: a stable sort on the (level,
    // octant) bits 35..42 keeps cells in order within each class (one pass;
    // the eighth below them never decreases in cell order within a level)
    radix_sort_u64(st.tkey.as<uint64_t>(), nullptr, st.tkey_alt.as<uint64_t>(), nullptr, ncell, 35, 43,
                   st.tmp.as<int32_t>(), s);
    m2l_count_targets(st.tkey.as<uint64_t>(), ncell, cnt + 2, s);
    Reader rd{a};
    rd.begin(cnt, 7 * 4, s);
    // while the host waits: the P2P leaves (by spatial eighth, costliest
    // first) and the cell centres, which need none of the sizes (unless
    // already built on another stream)
    if (!a.p2p_ready && !a.f64) build_p2p_leaves(st, a, s);
    int32_t h7[7];
    rd.end(h7, s);
    if (h7[5] > st.nslot_total) {
        if (a.f64) {
            const int64_t e64 = m2l_f64_op_elems(p);
            FMM_HIP_CHECK(st.frags64.grow_keep((size_t)h7[5] * e64 * 8, s));
            m2l_build_ops_f64(st.new_keys.as<int32_t>(), h7[6], st.slot_of.as<int32_t>(), p, e64, a.transposed,
                              st.frags64.as<double>(), s);
        } else {
            FMM_HIP_CHECK(st.frags.grow_keep((size_t)h7[5] * op_elems * 2, s));
            m2l_build_ops(st.new_keys.as<int32_t>(), h7[6], st.slot_of.as<int32_t>(), p, RT, op_elems, a.transposed,
                          st.frags.as<uint16_t>(), s);
        }
        st.nslot_total = h7[5];
    }
    if (h7[2] < 0 || h7[2] > ncell || h7[1] < 0 || h7[1] > npair || h7[5] < 0)
        throw std::runtime_error("M2L group build: device sizes out of range");
    st.nslot = h7[5];
    st.nextra = h7[1];
    st.ntarget = h7[2];
    st.ngroup = (st.ntarget + kGroupM2L - 1) / kGroupM2L;
    const int32_t ng = std::max(st.ngroup, 1);
    FMM_HIP_CHECK(st.gcount.grow((size_t)(ng + 1) * 4));
    FMM_HIP_CHECK(st.goff.grow((size_t)(ng + 1) * 4));
    FMM_HIP_CHECK(st.tcount.grow((size_t)(ng + 1) * 4));
    FMM_HIP_CHECK(st.toff.grow((size_t)(ng + 1) * 4));
    FMM_HIP_CHECK(st.gtarget.grow((size_t)ng * kGroupM2L * 4));
    FMM_HIP_CHECK(st.tmp.grow(std::max<size_t>(st.tmp.bytes, scan_tmp_elems(ng + 1) * 4)));
    const size_t gwords = (size_t)ng * ((st.nslot + 31) / 32 + 1);
    FMM_HIP_CHECK(st.gbits.grow(gwords * 4));
    FMM_HIP_CHECK(st.gwpre.grow(gwords * 4));
    const int chunk = std::max(1, std::min(kMaxTaskEntries, a.tuning.m2l_task_entries));
    m2l_group_count(st.tkey.as<uint64_t>(), st.ntarget, a.m2l_ptr, st.pcode.as<int32_t>(), st.slot_of.as<int32_t>(),
                    st.nslot, st.gbits.as<uint32_t>(), st.gwpre.as<uint32_t>(), st.gcount.as<int32_t>(), chunk,
                    st.tcount.as<int32_t>(), s);
    // entry and task offsets, their totals to cnt[3..4]; zeroes the per-XCD task counts cnt[16..24]
    m2l_group_scans(st.gcount.as<int32_t>(), st.tcount.as<int32_t>(), st.ngroup, st.goff.as<int32_t>(),
                    st.toff.as<int32_t>(), cnt + 3, cnt + 16, st.tmp.as<int32_t>(), s);
    rd.begin(cnt + 3, 8, s);
    // while the host waits: the pairs left to the per-pair kernel
    // (|delta| > kDeltaMax or far displacement), whose number is known
    FMM_HIP_CHECK(st.xsrc.grow((size_t)std::max(st.nextra, 1) * 4));
    m2l_extra(a.m2l_ptr, ncell, a.m2l_src, st.pcode.as<int32_t>(), st.xptr.as<int32_t>(), st.xsrc.as<int32_t>(), s);
    int32_t h2[2];
    rd.end(h2, s);
    if (h2[0] < 0 || h2[1] < 0 || (st.ngroup > 0 && (h2[0] < st.ngroup || h2[1] < st.ngroup)))
        throw std::runtime_error("M2L group build: entry or task count out of range");
    st.nentries = st.ngroup > 0 ? h2[0] : 0;
    st.ntask = st.ngroup > 0 ? h2[1] : 0;
    FMM_HIP_CHECK(st.ecls.grow((size_t)std::max(st.nentries, 1) * 4));
    FMM_HIP_CHECK(st.esrc.grow((size_t)std::max(st.nentries, 1) * kGroupM2L * 4));
    const size_t nt1 = (size_t)std::max(st.ntask, 1);
    FMM_HIP_CHECK(st.tasks.grow(nt1 * sizeof(int4)));
    FMM_HIP_CHECK(st.tasks_alt.grow(nt1 * sizeof(int4)));
    FMM_HIP_CHECK(st.tkeys.grow(nt1 * 8 * 2));
    FMM_HIP_CHECK(st.tidx.grow(nt1 * 4 * 2));
    FMM_HIP_CHECK(st.tmp.grow(std::max<size_t>(st.tmp.bytes, radix_tmp_elems(nt1) * 4)));
    m2l_group_fill(st.tkey.as<uint64_t>(), st.ntarget, a.m2l_ptr, a.m2l_src, st.pcode.as<int32_t>(),
                   st.slot_of.as<int32_t>(), st.nslot, st.gbits.as<uint32_t>(), st.gwpre.as<uint32_t>(),
                   st.goff.as<int32_t>(), st.gcount.as<int32_t>(), st.ecls.as<int32_t>(), st.esrc.as<int32_t>(),
                   st.gtarget.as<int32_t>(), s);
    m2l_make_tasks(st.gcount.as<int32_t>(), st.goff.as<int32_t>(), st.ngroup, chunk, std::max(st.nslot, 1),
                   st.toff.as<int32_t>(),
                   st.tkey.as<uint64_t>(), st.ntask, st.tasks.as<int4>(), st.tasks_alt.as<int4>(),
                   st.tkeys.as<uint64_t>(), st.tkeys.as<uint64_t>() + nt1, st.tidx.as<uint32_t>(),
                   st.tidx.as<uint32_t>() + nt1, cnt + 16, st.tmp.as<int32_t>(), s);
    st.f64 = a.f64;
    if (a.f64) {   // no work queue: the tasks are launched as a grid
        st.built = true;
        return;
    }
    // ---- the 16 task lists (M2L and P2P per XCD), built on the device
    if (a.p2p_ready) FMM_HIP_CHECK(hipStreamWaitEvent(s, a.p2p_ready, 0));
    FMM_HIP_CHECK(st.lists.grow(16 * sizeof(int4)));
    hipLaunchKernelGGL(k_make_lists, dim3(1), dim3(64), 0, s, cnt + 16, 0, st.lists.as<int4>());
    FMM_LAUNCH_CHECK();
    st.built = true;
}

void build_p2p_leaves(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    const int32_t ncell = a.ncell;
    FMM_HIP_CHECK(st.cnt.grow(64 * 4));   // the per-eighth leaf counts go to cnt[24 .. 32]
    FMM_HIP_CHECK(st.leafbuf.grow((size_t)4 * (ncell + 1) * 4));
    FMM_HIP_CHECK(st.leaves.grow((size_t)std::max(ncell, 1) * 4));
    FMM_HIP_CHECK(st.tmp2.grow(radix_tmp_elems(ncell) * 4));
    p2p_leaf_list(a.g.c, ncell, a.n, a.p2p_ptr, a.p2p_src, a.leaf_cost, st.leafbuf.as<int32_t>(),
                  st.leaves.as<int32_t>(), st.tmp2.as<int32_t>(), st.cnt.as<int32_t>() + 24, s);
    // the P2P task lists (the M2L ones follow from the far-field build)
    FMM_HIP_CHECK(st.lists.grow(16 * sizeof(int4)));
    hipLaunchKernelGGL(k_make_lists, dim3(1), dim3(64), 0, s, st.cnt.as<int32_t>() + 25, 1, st.lists.as<int4>());
    FMM_LAUNCH_CHECK();
    // the cell centres, which the P2P tasks read (target and source leaf offsets)
    FMM_HIP_CHECK(st.centre.grow((size_t)std::max(ncell, 1) * 3 * 8));
    cell_centres(a.g, ncell, st.centre.as<double>(), s);
}

void reorder_p2p_leaves(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    if (!st.built || st.f64) return;
    build_p2p_leaves(st, a, s);
}

void near_far_prepare(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    if (!st.built) throw std::runtime_error("mixed near/far stage used before its build");
    if (a.n > 0 && (!a.M || !a.L || !a.phi || !a.fld || !a.qs))
        throw std::runtime_error("mixed near/far stage: an input or output workspace is missing");
    const int P = ncoef(a.p);
    const int32_t ncell = a.ncell;
    FMM_HIP_CHECK(st.M32.grow((size_t)(ncell + 1) * queue_mrow_elems(a.p) * 2));
    FMM_HIP_CHECK(st.pf.grow((size_t)std::max<int64_t>(a.n, 1) * sizeof(float4)));
    FMM_HIP_CHECK(st.cnt.grow(64 * 4));
    FMM_HIP_CHECK(st.part.grow((size_t)std::max(st.ntask, 1) * queue_part_elems(a.p) * sizeof(float)));
    queue_split_multipoles(a.M, ncell, a.p, st.M32.as<uint16_t>(), s);
    fill_zero(a.L, (size_t)ncell * P * 8, s);
    if (!st.early) p2p_prepare(a.g, a.n, a.leaf_of, a.xs, a.ys, a.zs, a.qs, st.pf.as<float4>(), s);
}

namespace {

void ensure_streams(NearFarState &st) {
    if (st.side) return;
    // default priority, like the plan's stream
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&st.side, hipStreamNonBlocking));
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&st.side2, hipStreamNonBlocking));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&st.fork, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&st.join, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&st.after_queue, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&st.after_side, hipEventDisableTiming));
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&st.side3, hipStreamNonBlocking));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&st.early_fork, hipEventDisableTiming));
    FMM_HIP_CHECK(hipEventCreateWithFlags(&st.early_done, hipEventDisableTiming));
}

int compute_units() {
    int dev = 0, ncu = 256;
    FMM_HIP_CHECK(hipGetDevice(&dev));
    FMM_HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    return ncu;
}

// with_side / with_early: this queue's side kernel, an early P2P kernel
QueueStreams streams_of(const NearFarState &st, bool with_side, bool with_early) {
    QueueStreams qs;
    qs.side = with_side ? st.side : nullptr;
    qs.side2 = st.side2;
    qs.fork = st.fork;
    qs.join = st.join;
    qs.after_queue = st.after_queue;
    qs.after_side = st.after_side;
    qs.early = with_early ? st.side3 : nullptr;
    qs.early_done = st.early_done;
    return qs;
}

QueueArgs queue_args(NearFarState &st, const NearFarArgs &a) {
    const int32_t ncell = a.ncell;
    QueueArgs q;
    q.c = a.g.c;
    q.centre = st.centre.as<double>();
    q.m2l_tasks = st.tasks.as<int4>();
    q.gtarget = st.gtarget.as<int32_t>();
    q.ecls = st.ecls.as<int32_t>();
    q.esrc = st.esrc.as<int32_t>();
    q.ops = st.frags.as<uint16_t>();
    q.Mb = st.M32.as<uint16_t>();
    q.zero_row = ncell;
    q.part = st.part.as<float>();
    q.P = ncoef(a.p);
    q.toff = st.toff.as<int32_t>();
    q.tcount = st.tcount.as<int32_t>();
    q.ngroup = st.ntask > 0 ? st.ngroup : 0;
    q.L = a.L;
    q.leaves = st.leaves.as<int32_t>();
    q.p2p_ptr = a.p2p_ptr;
    q.p2p_src = a.p2p_src;
    q.pf = st.pf.as<float4>();
    q.phi = a.phi;
    q.fld = a.fld;
    q.lists = st.lists.as<int4>();
    q.heads = a.heads ? a.heads : st.cnt.as<int32_t>() + 40;
    q.trace = a.trace && a.trace_count && a.trace_cap > 0 ? a.trace : nullptr;
    q.trace_count = a.trace_count;
    q.trace_cap = a.trace_cap;
    q.leaf_cost = a.cost_out;
    return q;
}

}  // namespace

bool near_far_start_p2p(NearFarState &st, const NearFarArgs &a, hipStream_t from) {
    near_far_drop_early(st, from);
    const int side_per_cu = std::max(0, std::min(8, a.tuning.p2p_per_cu));
    const int early_per_cu = std::max(0, std::min(side_per_cu, a.tuning.early_p2p_per_cu));
    if (early_per_cu == 0 || a.trace || a.n <= 0 || st.f64) return false;
    if (!a.phi || !a.fld || !a.qs || !st.leaves.ptr || !st.lists.ptr || !st.centre.ptr || !st.cnt.ptr)
        throw std::runtime_error("early near field: inputs or outputs not prepared");
    ensure_streams(st);
    FMM_HIP_CHECK(st.pf.grow((size_t)a.n * sizeof(float4)));
    QueueArgs q = queue_args(st, a);
    // on `from`, so that whatever follows it (the k_queue that later claims
    // the M2L tasks) sees the counters zeroed
    fill_zero(q.heads, 16 * sizeof(int32_t), from);
    FMM_HIP_CHECK(hipEventRecord(st.early_fork, from));
    FMM_HIP_CHECK(hipStreamWaitEvent(st.side3, st.early_fork, 0));
    p2p_prepare(a.g, a.n, a.leaf_of, a.xs, a.ys, a.zs, a.qs, st.pf.as<float4>(), st.side3);
    st.early_wg = compute_units() * early_per_cu;
    queue_p2p_start(q, st.early_wg, st.side3);
    st.early = true;
    st.early_heads = q.heads;
    return true;
}

void near_far_drop_early(NearFarState &st, hipStream_t s) {
    if (!st.early) return;
    FMM_HIP_CHECK(hipEventRecord(st.early_done, st.side3));
    FMM_HIP_CHECK(hipStreamWaitEvent(s, st.early_done, 0));
    st.early = false;
    st.early_heads = nullptr;
}

bool near_far_queue(NearFarState &st, const NearFarArgs &a, hipStream_t s, bool defer_join, bool *joined_early) {
    if (joined_early) *joined_early = false;
    if (!st.built) throw std::runtime_error("mixed near/far stage used before its build");
    if (a.n > 0 && (!a.L || !a.phi || !a.fld || !st.M32.ptr || !st.pf.ptr || !st.centre.ptr || !st.leaves.ptr ||
                    !st.lists.ptr || (st.ntask > 0 && st.part.bytes < (size_t)st.ntask * queue_part_elems(a.p) * 4)))
        throw std::runtime_error("mixed near/far stage: queue inputs not prepared");
    QueueArgs q = queue_args(st, a);
    // an early P2P kernel with other claim counters (or without room for
    // it in this launch shape) is waited for and the near field recomputed
    if (st.early && (st.early_heads != q.heads || q.trace)) near_far_drop_early(st, s);
    const bool side_running = st.early;
    if (q.trace) fill_zero(a.trace_count, sizeof(int32_t), s);
    const int ncu = compute_units();
    const int per_cu = std::max(1, std::min(8, a.tuning.grid_per_cu));
    const int side_per_cu = std::max(0, std::min(8, a.tuning.p2p_per_cu));
    // the side workgroups not started early
    const int nside = std::max(0, ncu * side_per_cu - (side_running ? st.early_wg : 0));
    if (nside > 0 || side_running) ensure_streams(st);
    QueueStreams qs = streams_of(st, nside > 0, side_running);
    const bool deferred = queue_run(q, a.p, ncu * per_cu, nside, qs, s, defer_join);
    st.tail_pending = deferred;
    st.tail_side = nside > 0;
    st.tail_early = side_running;
    st.early = false;   // joined by this queue from now on
    st.early_heads = nullptr;
    if (joined_early) *joined_early = side_running;
    return deferred;
}

void near_far_tail(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    if (!st.tail_pending) return;
    const int per_cu = std::max(1, std::min(8, a.tuning.grid_per_cu));
    queue_tail(queue_args(st, a), compute_units() * per_cu, streams_of(st, st.tail_side, st.tail_early), s);
    st.tail_pending = false;
}

void near_far_join(NearFarState &st, hipStream_t s) {
    if (st.tail_pending) throw std::runtime_error("work queue joined before its P2P tail was launched");
    FMM_HIP_CHECK(hipStreamWaitEvent(s, st.join, 0));
}

hipStream_t near_far_join_stream(const NearFarState &st) { return st.side2; }

void near_far_rest(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    if (st.nextra <= 0) return;
    if (a.transposed)
        launch_m2l_fp64_adjoint(a.g, a.ncell, a.p, st.xptr.as<int32_t>(), st.xsrc.as<int32_t>(), st.nextra, a.M, a.L,
                                1, a.deterministic, s);
    else
        launch_m2l_fp64_add(a.g, a.ncell, a.p, st.xptr.as<int32_t>(), st.xsrc.as<int32_t>(), st.nextra, a.M, a.L,
                            a.deterministic, s);
}

void m2l_f64_run(NearFarState &st, const NearFarArgs &a, hipStream_t s) {
    if (!st.built || !st.f64) throw std::runtime_error("FP64 M2L tables not built");
    const int P = ncoef(a.p);
    FMM_HIP_CHECK(st.part64.grow((size_t)std::max(st.ntask, 1) * P * kGroupM2L * sizeof(double)));
    fill_zero(a.L, (size_t)a.ncell * P * sizeof(double), s);
    m2l_f64_tasks(st.tasks.as<int4>(), st.ntask, st.ecls.as<int32_t>(), st.esrc.as<int32_t>(), st.frags64.as<double>(),
                  a.M, a.p, st.part64.as<double>(), s);
    reduce_partials_f64(st.part64.as<double>(), st.toff.as<int32_t>(), st.tcount.as<int32_t>(),
                        st.gtarget.as<int32_t>(), st.ntask > 0 ? st.ngroup : 0, a.p, a.L, s);
    near_far_rest(st, a, s);
}

void release_near_far(NearFarState &st) {
    DevBuf *all[] = {&st.used, &st.slot_of, &st.nslots, &st.new_keys, &st.frags, &st.pcode, &st.xcount, &st.tkey,
                     &st.tkey_alt, &st.has, &st.gcount, &st.goff, &st.tcount, &st.toff, &st.ecls, &st.esrc, &st.gtarget, &st.tasks,
                     &st.xsrc, &st.xptr, &st.leafbuf, &st.leaves, &st.pf, &st.M32, &st.tmp, &st.cnt, &st.centre, &st.gbits, &st.gwpre, &st.tasks_alt, &st.tkeys, &st.tidx, &st.lists, &st.tmp2, &st.part, &st.key_rank, &st.frags64, &st.part64};
    if (st.side) {   // the side kernels may still read these buffers
        (void)hipStreamSynchronize(st.side);
        (void)hipStreamSynchronize(st.side2);
        (void)hipStreamSynchronize(st.side3);
    }
    for (DevBuf *b : all) b->release();
    if (st.side) {
        (void)hipStreamDestroy(st.side);
        (void)hipStreamDestroy(st.side2);
        (void)hipEventDestroy(st.fork);
        (void)hipEventDestroy(st.join);
        (void)hipEventDestroy(st.after_queue);
        (void)hipEventDestroy(st.after_side);
        (void)hipStreamDestroy(st.side3);
        (void)hipEventDestroy(st.early_fork);
        (void)hipEventDestroy(st.early_done);
    }
    st.early = false;
    st.early_heads = nullptr;
    st.side = st.side2 = st.side3 = nullptr;
    st.fork = st.join = st.after_queue = st.after_side = st.early_fork = st.early_done = nullptr;
    st.p = -1;
    st.built = false;
}

}  // namespace fmm
