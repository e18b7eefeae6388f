// steps.hip -- dataflow-scheduled sparse LU and substitutions in LDS, one
// workgroup per Jacobian, for gfx950.
//
// Every entry of the factors and of the RHS is an fma chain with a fixed
// order (Sec. 2 / Alg. 1 steps 2-3 realised without pivoting):
//   u_jj, u_jm, l_ij   updates l_ik u_kj over k in R_i ^ R_j ascending
//                      (l_ij divided by u_jj at the end);
//   forward  y_i       updates l_ik y_k, k ascending (column-oriented order);
//   backward y_i       updates u_ij x_j, j descending, then x_i = y_i / u_ii.
// The level schedule waits for whole etree levels and then runs each chain in
// one go; its critical path is the sum over levels of the longest chain of
// the level.  Here each update is placed at the earliest barrier step at which
// both of its inputs are final and all earlier updates of the same chain have
// run, so chains advance while their inputs are still being produced.  The
// per-entry operations and their order are unchanged, so the results equal
// the reference bit for bit; only the interleaving across entries differs.
// Forward substitution shares the factor's timeline (y_i needs only the final
// l_ik and y_k); backward substitution follows it.
//
// Host side: the schedule is built once per plan (a few hundred thousand
// tasks at n ~ 1000).  A task is one run of consecutive chain updates of one
// entry within one step, optionally ending with the division.  Thread t of the
// workgroup runs task t of a step; a step with more tasks than threads is
// split into consecutive sub-steps.  A step's descriptors are contiguous, one
// coalesced 16-byte load per lane, issued several steps ahead: a step itself is
// a few hundred cycles of LDS work, far less than one round trip to L2.
//
// Descriptor (int4, 16 bytes), LDS indices < 2^15 - 1, at most kStSegMax = 3
// updates per task:
//   x = dst | cnt << 15 | div << 17   (cnt 0..3; div = 0x7FFF: no division)
//   y, z, w = update pairs a | b << 16, in chain order (unused: 0); in a packed
//             schedule bit 15 of y marks a task that starts from 0, not v[dst]
// An empty slot has x = -1.  Update of a pair: v[dst] = fma(-v[a], v[b], v[dst]).
//
// Device side: LDS holds [u_jj (n) | L values (nnzL) | U values (nnzL) |
// y (n) | combine accumulator (n)] in doubles; one workgroup takes a Jacobian,
// runs its K perturbed systems one after the other and accumulates
// sum_k c_k x_k in the order of the reference combine (ascending k, fma chain
// from 0).
//
// Packed schedules.  A step is a few hundred cycles of dependent LDS work and a
// barrier, so a CU runs two workgroups' steps far faster than one's: at n = 601
// two resident workgroups per CU take 512 Jacobians in 0.77 ms instead of
// 1.11 ms.  That needs at most 80 KB of LDS per workgroup (and registers for
// eight waves per SIMD); unpacked, n = 601 needs 103 KB, and n = 1,001 does not
// fit at all.  An L or U value needs LDS only from its gather (an
// entry of A, or a value never written, which reads as 0) or its first write,
// to its last read; a fill value's first task can start from zero instead of
// reading its slot.  The values are packed into a pool of shared slots by these
// live intervals in executed steps (greedy by start time, which uses exactly as
// many slots as values are live at the busiest step: 16,095 instead of 21,728
// at n = 1,001; 7,651 instead of 11,016 at n = 601), and a slot is reused only
// in a step after its previous value's last read, so no step reads a slot that
// a task of the step writes.  The layout becomes [u_jj | pool | y | combine
// accumulator].  A pattern is packed when that brings it to two workgroups per
// CU or is the only way to fit; otherwise it keeps the plain layout.
#include <algorithm>
#include <climits>
#include <queue>
#include <vector>

#include "dense.h"
#include "sparse.h"

namespace psp {

namespace {
constexpr int kStThreads = 1024;         // workgroup size; the schedule is built for it (one task per thread and step)
constexpr int kStAhead = 7;              // steps whose descriptors are in flight
constexpr int kStRingShort = 4;          // the shallower ring the tuner may choose
// Longest run of one chain inside a step, so that every task's updates fit in
// its descriptor (no second, dependent load).  The long runs belong mostly to
// the dense slack row, whose value is needed only at the end; at n = 601 the
// cap raises the step count from 294 to 340 and removes every in-step fetch.
constexpr int kStSegMax = 3;
constexpr int kStLdsLimit = 152 * 1024;  // bytes of LDS the kernel may use
// Static LDS of the kernel (pivot flag, nodes and weights: 260 bytes, 272 as
// allocated), reserved with margin; steps_run checks the compiled figure
// against it before the first launch.
constexpr int64_t kStStaticLds = 512;
constexpr int64_t kStLdsPair = 80 * 1024 - kStStaticLds;   // dynamic LDS at most this: two workgroups share a CU

// Values in the unpacked layout (the index space the schedule is built in).
int64_t st_lds_doubles(const Symbolic& s) { return 3 * (int64_t)s.n + 2 * (int64_t)s.l_ptr[s.n]; }
constexpr int64_t kStLdsMax = 160 * 1024 - kStStaticLds;   // dynamic LDS: values + per-step metadata
// bytes: [u_jj | L and U values (pool) | y | cx] rounded to 16 B, then one int2 of metadata per
// padded step and ring slot
__host__ __device__ constexpr int st_padded(int S) { return (S + kStAhead - 1) / kStAhead * kStAhead; }
int64_t st_lds_total(int64_t n, int64_t pool, int64_t S) {
    return ((3 * n + pool + 1) & ~1LL) * 8 + 8 * ((int64_t)st_padded((int)S) + kStAhead + 1);
}

struct StTask {
    int32_t step, dst, div, off, cnt;
};

// Packs the L and U values of a built schedule (unpacked indices, see above)
// into shared LDS slots by live interval, rewriting every descriptor.
bool pack_slots(const Symbolic& s, const std::vector<int32_t>& meta, std::vector<int32_t>& desc, int S,
                std::vector<int32_t>& slot_l, std::vector<int32_t>& slot_u, int32_t& pool) {
    const int n = s.n, nl = s.l_ptr[n], P0 = 2 * nl;
    // entries of A land in L / U positions by the gather; everything else starts unwritten
    std::vector<char> inA(P0, 0);
    auto pos_in_col = [&](int col, int row) {
        const int* b0 = s.l_idx.data() + s.l_ptr[col];
        const int* e0 = s.l_idx.data() + s.l_ptr[col + 1];
        const int* q = std::lower_bound(b0, e0, row);
        return (q != e0 && *q == row) ? (int)(q - s.l_idx.data()) : -1;
    };
    for (int r = 0; r < n; ++r)
        for (int e = s.row_ptr[r]; e < s.row_ptr[r + 1]; ++e) {
            const int pr = s.iperm[r], pc = s.iperm[s.col_idx[e]];
            const int t = pr > pc ? pos_in_col(pc, pr) : (pr < pc ? pos_in_col(pr, pc) : -1);
            if (t >= 0) inA[(pr > pc ? 0 : nl) + t] = 1;
        }
    auto pooled = [&](int i) { return i >= n && i < n + P0; };
    std::vector<int> first(P0, INT_MAX), last(P0, -1);
    for (int st = 0; st < S; ++st) {
        const int base = meta[4 * st], tact = meta[4 * st + 1];
        for (int t = 0; t < tact; ++t) {
            const int32_t* d = &desc[4 * (size_t)(base + t)];
            if (d[0] == -1) continue;
            const int dst = d[0] & 0x7FFF, cnt = (d[0] >> 15) & 3, div = (int)((uint32_t)d[0] >> 17);
            if (pooled(dst)) {
                first[dst - n] = std::min(first[dst - n], st);
                last[dst - n] = std::max(last[dst - n], st);
            }
            for (int c = 0; c < cnt; ++c) {
                const uint32_t w = (uint32_t)d[1 + c];
                const int a = (int)(w & 0xFFFF), b = (int)(w >> 16);
                if (pooled(a)) last[a - n] = std::max(last[a - n], st);
                if (pooled(b)) last[b - n] = std::max(last[b - n], st);
            }
            if (div != 0x7FFF && pooled(div)) last[div - n] = std::max(last[div - n], st);
        }
    }
    // live interval [birth, last]: birth -1 for gathered values
    std::vector<int> birth(P0), order(P0), slot(P0, -1);
    for (int i = 0; i < P0; ++i) {
        birth[i] = (inA[i] || first[i] == INT_MAX) ? -1 : first[i];
        last[i] = std::max(last[i], birth[i]);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return birth[a] < birth[b]; });
    std::priority_queue<std::pair<int, int>, std::vector<std::pair<int, int>>, std::greater<std::pair<int, int>>> active;
    std::priority_queue<int, std::vector<int>, std::greater<int>> freed;
    int used = 0;
    for (int i : order) {
        while (!active.empty() && active.top().first < birth[i]) {
            freed.push(active.top().second);
            active.pop();
        }
        int sl = used;
        if (!freed.empty()) {
            sl = freed.top();
            freed.pop();
        } else {
            ++used;
        }
        slot[i] = sl;
        active.push({last[i], sl});
    }
    if (3 * n + used >= 0x7FFF) return false;
    auto remap = [&](int i) { return i < n ? i : (i < n + P0 ? n + slot[i - n] : i - P0 + used); };
    for (int st = 0; st < S; ++st) {
        const int base = meta[4 * st], tact = meta[4 * st + 1];
        for (int t = 0; t < tact; ++t) {
            int32_t* d = &desc[4 * (size_t)(base + t)];
            if (d[0] == -1) continue;
            const int dst = d[0] & 0x7FFF, cnt = (d[0] >> 15) & 3, div = (int)((uint32_t)d[0] >> 17);
            const uint32_t zero = (pooled(dst) && birth[dst - n] == st) ? 1u : 0u;
            const uint32_t nd = div == 0x7FFF ? 0x7FFFu : (uint32_t)remap(div);
            d[0] = (int32_t)((uint32_t)remap(dst) | ((uint32_t)cnt << 15) | (nd << 17));
            for (int c = 0; c < cnt; ++c) {
                const uint32_t w = (uint32_t)d[1 + c];
                d[1 + c] = (int32_t)((uint32_t)remap((int)(w & 0xFFFF)) | ((uint32_t)remap((int)(w >> 16)) << 16));
            }
            d[1] = (int32_t)((uint32_t)d[1] | (zero << 15));
        }
    }
    for (int t = 0; t < nl; ++t) {
        slot_l[t] = birth[t] < 0 ? n + slot[t] : -1;
        slot_u[t] = birth[nl + t] < 0 ? n + slot[nl + t] : -1;
    }
    pool = used;
    return true;
}

// Builds the step schedule.  Returns false when the plan does not fit.
bool build_schedule(const Symbolic& s, const std::vector<int32_t>& r_pos, int T, std::vector<int32_t>& meta,
                    std::vector<int32_t>& desc, int32_t& nsteps, bool pack, std::vector<int32_t>& slot_l,
                    std::vector<int32_t>& slot_u, int32_t& pool, int seg_max = kStSegMax) {
    const int n = s.n, nl = s.l_ptr[n];
    if (st_lds_doubles(s) >= 0x7FFF) return false;
    if (!pack && st_lds_doubles(s) * 8 > kStLdsLimit) return false;
    const int ybase = n + 2 * nl;
    auto LX = [&](int t) { return n + t; };
    auto UX = [&](int t) { return n + nl + t; };
    auto YX = [&](int i) { return ybase + i; };
    auto pk = [](int a, int b) { return (uint32_t)a | ((uint32_t)b << 16); };

    std::vector<int32_t> fin(ybase + n, 0);   // step after which an entry holds its final value (0: gathered)
    std::vector<uint32_t> P;                  // all updates, grouped by task
    std::vector<StTask> tasks;
    std::vector<uint32_t> chain;

    // Splits the chain of `dst` (in `chain`, in order) into steps; base: first step - 1.
    auto place = [&](int dst, int div, int base) {
        int seg_step = -1, seg_cnt = 0;
        int64_t seg_off = 0;
        for (uint32_t q : chain) {
            const int a = (int)(q & 0xFFFF), b = (int)(q >> 16);
            const int ready = std::max(std::max(fin[a], fin[b]), base) + 1;
            int stp = std::max(ready, seg_step);
            if (stp == seg_step && seg_cnt == seg_max) stp = seg_step + 1;   // long runs continue next step
            if (stp != seg_step) {
                if (seg_cnt) tasks.push_back({seg_step, dst, -1, (int32_t)seg_off, seg_cnt});
                seg_step = stp;
                seg_off = (int64_t)P.size();
                seg_cnt = 0;
            }
            P.push_back(q);
            ++seg_cnt;
        }
        if (seg_cnt) tasks.push_back({seg_step, dst, -1, (int32_t)seg_off, seg_cnt});
        int last = seg_cnt ? seg_step : -1;
        if (div >= 0) {
            const int need = std::max(fin[div], base) + 1;
            if (seg_cnt && seg_step >= need) {
                tasks.back().div = div;
            } else {
                tasks.push_back({need, dst, div, 0, 0});
                last = need;
            }
        }
        if (last >= 0) fin[dst] = last;
    };
    // (l at pos(a,k), u at pos(b,k)) for k in R_a ^ R_b ascending
    auto merge = [&](int a, int b) {
        int p = s.lrow_ptr[a], pe = s.lrow_ptr[a + 1], q = s.lrow_ptr[b], qe = s.lrow_ptr[b + 1];
        while (p < pe && q < qe) {
            const int ka = s.lrow_idx[p], kb = s.lrow_idx[q];
            if (ka == kb) {
                chain.push_back(pk(LX(r_pos[p]), UX(r_pos[q])));
                ++p;
                ++q;
            } else if (ka < kb) {
                ++p;
            } else {
                ++q;
            }
        }
    };
    // factor, column by column (every input of column j lies in earlier columns)
    for (int j = 0; j < n; ++j) {
        chain.clear();
        for (int p = s.lrow_ptr[j]; p < s.lrow_ptr[j + 1]; ++p) chain.push_back(pk(LX(r_pos[p]), UX(r_pos[p])));
        place(j, -1, 0);
        for (int t = s.l_ptr[j]; t < s.l_ptr[j + 1]; ++t) {
            const int m = s.l_idx[t];
            chain.clear();
            merge(j, m);     // u_jm: l_jk u_km
            place(UX(t), -1, 0);
            chain.clear();
            merge(m, j);     // l_mj: l_mk u_kj, then / u_jj
            place(LX(t), j, 0);
        }
    }
    // forward substitution on the same timeline
    for (int i = 0; i < n; ++i) {
        chain.clear();
        for (int p = s.lrow_ptr[i]; p < s.lrow_ptr[i + 1]; ++p) chain.push_back(pk(LX(r_pos[p]), YX(s.lrow_idx[p])));
        place(YX(i), -1, 0);
    }
    int s1 = 0;
    for (const StTask& t : tasks) s1 = std::max(s1, t.step);
    // backward substitution after it: row i of U has the pattern of column i of L
    for (int i = n - 1; i >= 0; --i) {
        chain.clear();
        for (int t = s.l_ptr[i + 1] - 1; t >= s.l_ptr[i]; --t) chain.push_back(pk(UX(t), YX(s.l_idx[t])));
        place(YX(i), i, s1);
    }
    int S = 0;
    for (const StTask& t : tasks) S = std::max(S, t.step);

    // Group by step; a step with more tasks than threads becomes consecutive
    // sub-steps (its tasks are independent), longest tasks first so that
    // the long ones share a sub-step.  Thread t runs task t of its sub-step.
    std::vector<std::vector<int32_t>> by_step(S + 1);
    for (int32_t i = 0; i < (int32_t)tasks.size(); ++i) by_step[tasks[i].step].push_back(i);
    meta.clear();
    desc.clear();
    auto cost = [&](const StTask& t) { return 6 + 2 * t.cnt + (t.div >= 0 ? 8 : 0); };
    for (int st = 1; st <= S; ++st) {
        std::vector<int32_t>& list = by_step[st];
        std::stable_sort(list.begin(), list.end(),
                         [&](int32_t a, int32_t b) { return cost(tasks[a]) > cost(tasks[b]); });
        for (size_t c0 = 0; c0 < list.size(); c0 += (size_t)T) {
            const int cnt = (int)std::min<size_t>((size_t)T, list.size() - c0);
            const int tact = (cnt + 63) / 64 * 64;
            const int64_t base = (int64_t)desc.size() / 4;
            if (base + tact > INT_MAX / 2) return false;
            meta.push_back((int32_t)base);
            meta.push_back(tact);
            meta.push_back(1);
            meta.push_back(0);
            desc.resize(desc.size() + 4 * (size_t)tact, 0);
            for (int t = cnt; t < tact; ++t) desc[4 * (size_t)(base + t)] = -1;
            for (int t = 0; t < cnt; ++t) {
                const StTask& k = tasks[list[c0 + t]];
                if (k.cnt > 3) return false;
                const size_t at = 4 * (size_t)(base + t);
                desc[at] = (int32_t)((uint32_t)k.dst | ((uint32_t)k.cnt << 15) |
                                     ((uint32_t)(k.div >= 0 ? k.div : 0x7FFF) << 17));
                for (int c = 0; c < k.cnt; ++c) desc[at + 1 + c] = (int32_t)P[k.off + c];
            }
        }
    }
    S = (int)(meta.size() / 4);
    slot_l.resize(nl);
    slot_u.resize(nl);
    if (!pack) {
        for (int t = 0; t < nl; ++t) {
            slot_l[t] = n + t;
            slot_u[t] = n + nl + t;
        }
        pool = 2 * nl;
    } else if (!pack_slots(s, meta, desc, S, slot_l, slot_u, pool)) {
        return false;
    }
    if ((3 * (int64_t)n + pool) * 8 > kStLdsLimit || st_lds_total(n, pool, S) > kStLdsMax) return false;
    nsteps = S;
    return true;
}

struct StArgs {
    StepIdx sx;
    SpIdx ix;
    int32_t nnz, batch, K, per_jacobian;
    const double* values;   // batch x nnz
    const double* dvec;
    const double* B;        // batch x n
    double* X;              // batch x n        (per_jacobian)
    double* Xk;             // batch x K x n    (otherwise; per_jacobian: also written when xk_too)
    int32_t* info;          // batch x K
    int32_t xk_too;
    // list mode (per system): only the Jacobians list[0 .. *count-1], with nodes scale[s] eps_k
    const int32_t* list;
    const int32_t* count;
    const double* scale;
};

template <bool PACKED>
__device__ __forceinline__ void st_exec(double* v, int4 d) {
    if (d.x == -1) return;
    const int dst = d.x & 0x7FFF;
    const int cnt = (d.x >> 15) & 3;
    const int div = (int)((uint32_t)d.x >> 17);
    // The operands of every pair that some lane of the wave uses are read up front (unused
    // pairs of a lane read slot 0), pairs no lane of the wave uses are skipped by uniform
    // branches, and the chain selects instead of branching.  LDS instructions are what a
    // step spends most on: reading every pair in every wave cost 8 % of the kernel's time,
    // reading the divisor up front in every wave 7 %.
    const double a0 = v[dst];
    const double l0 = v[d.y & 0x7FFF], u0 = v[(uint32_t)d.y >> 16];
    double l1 = 0.0, u1 = 0.0, l2 = 0.0, u2 = 0.0;
    if (__builtin_amdgcn_ballot_w64(cnt > 1)) {
        l1 = v[d.z & 0xFFFF];
        u1 = v[(uint32_t)d.z >> 16];
    }
    if (__builtin_amdgcn_ballot_w64(cnt > 2)) {
        l2 = v[d.w & 0xFFFF];
        u2 = v[(uint32_t)d.w >> 16];
    }
    double acc = (PACKED && ((d.y >> 15) & 1)) ? 0.0 : a0;
    const double f0 = fmad(-l0, u0, acc);
    acc = cnt > 0 ? f0 : acc;
    const double f1 = fmad(-l1, u1, acc);
    acc = cnt > 1 ? f1 : acc;
    const double f2 = fmad(-l2, u2, acc);
    acc = cnt > 2 ? f2 : acc;
    // the division only in waves that have one (a uniform branch)
    const bool hd = div != 0x7FFF;
    if (__builtin_amdgcn_ballot_w64(hd)) {
        const double q = acc / v[hd ? div : 0];
        acc = hd ? q : acc;
    }
    v[dst] = acc;
}

// Descriptor of thread tid in a step, through a bounds-checked buffer load:
// threads past the step's active count pass an out-of-range offset, which
// returns zeros without a memory access.  (A plain load from a shared dummy
// slot sends every idle lane of every CU to one cache line at once.)  The
// instruction is issued by every thread, so the loads in flight stay static.
__device__ __forceinline__ int4 st_desc(__amdgpu_buffer_rsrc_t r, int2 m, int tid) {
    const int off = tid < m.y ? (m.x + tid) * 16 : -1;
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    int4 d;
    __builtin_memcpy(&d, &w, sizeof(d));
    return d;
}

// waves_per_eu(8): registers for eight waves per SIMD, i.e. two 1024-lane workgroups per CU
// (without it the kernel takes 112 scalar registers per wave, which leaves room for seven)
// RING: steps whose descriptors are in flight (kStAhead, or a shallower ring that the tuner may pick);
// the metadata LDS is sized for kStAhead, which covers every shallower ring.
template <int T, bool PACKED, bool LIST, int RING>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(8))) void steps_kernel(StArgs a, EpsSet es) {
    // 16-byte aligned: the step metadata after the values is read as int4
    // (a misaligned ds_read_b128 every step costs several times the step)
    extern __shared__ __align__(16) double v[];
    __shared__ int s_bad;
    // the nodes and weights, read once per system: kept in LDS, not in scalar registers
    // for the whole kernel (which would cost eight-wave occupancy)
    __shared__ double s_eps[kMaxK], s_c[kMaxK];
    const SpIdx& ix = a.ix;
    const int n = ix.n, nl = ix.nnzl, tid = threadIdx.x;
    const int ybase = n + a.sx.pool;
    double* y = v + ybase;
    double* cx = y + n;
    const int S = a.sx.nsteps;
    const int Sp = (S + RING - 1) / RING * RING;
    // per-step metadata, read by every step of every system: kept in LDS,
    // followed by empty steps up to a multiple of the ring depth and one ring beyond
    int2* sm = reinterpret_cast<int2*>(v + ((3 * n + a.sx.pool + 1) & ~1));
    for (int i = tid; i < Sp + RING + 1; i += T) {
        const int4 mi = i < S ? a.sx.meta[i] : make_int4(0, 0, 1, 0);
        sm[i] = make_int2(mi.x, mi.y);
    }
#pragma unroll
    for (int i = 0; i < kMaxK; ++i)
        if (tid == i) {
            s_eps[i] = es.eps[i];
            s_c[i] = es.c[i];
        }
    __syncthreads();
    // gfx9-family buffer resource: raw (stride 0), range = the descriptor array
    const __amdgpu_buffer_rsrc_t drs =
        __builtin_amdgcn_make_buffer_rsrc((void*)a.sx.desc, (short)0, a.sx.ndesc * 16, 0x00020000);
    const int njobs = LIST ? *a.count * es.K : (a.per_jacobian ? a.batch : a.batch * es.K);
    for (int job = blockIdx.x; job < njobs; job += gridDim.x) {
        const int s = LIST ? a.list[job / es.K] : (a.per_jacobian ? job : job / es.K);
        const int k0 = a.per_jacobian ? 0 : job % es.K, k1 = a.per_jacobian ? es.K : k0 + 1;
        const double* vals = a.values + (int64_t)s * a.nnz;
        for (int kk = k0; kk < k1; ++kk) {
            // descriptor ring: step st runs while steps st+1 .. st+RING-1 are in
            // flight; each step waits for its own load only.
            int4 ring[RING];
#pragma unroll
            for (int d = 0; d < RING; ++d) {
                ring[d] = st_desc(drs, sm[d], tid);
            }
            int2 m = sm[0];
            // A + eps_k D permuted onto the fill pattern, and P b (packed: only the
            // values live from the start; fill values start from zero at their first task)
            for (int t = tid; t < nl; t += T) {
                const int sl = ix.src_l[t], su = ix.src_u[t];
                if (!PACKED) {
                    v[n + t] = sl >= 0 ? vals[sl] : 0.0;
                    v[n + nl + t] = su >= 0 ? vals[su] : 0.0;
                } else {
                    const int dl = a.sx.slot_l[t], du = a.sx.slot_u[t];
                    if (dl >= 0) v[dl] = sl >= 0 ? vals[sl] : 0.0;
                    if (du >= 0) v[du] = su >= 0 ? vals[su] : 0.0;
                }
            }
            // a power-of-two node scale (list mode) multiplies every node exactly
            const double ek = LIST ? __dmul_rn(s_eps[kk], a.scale[s]) : s_eps[kk];
            for (int j = tid; j < n; j += T) {
                const int sd = ix.src_d[j], pj = ix.perm[j];
                const double ajj = sd >= 0 ? vals[sd] : 0.0;
                v[j] = __dadd_rn(ajj, __dmul_rn(ek, a.dvec ? a.dvec[pj] : 1.0));
                y[j] = a.B[(int64_t)s * n + pj];
            }
            if (tid == 0) s_bad = INT_MAX;
            __syncthreads();
            // No guard inside the rotation (the padded steps have no tasks): a
            // conditional here makes the compiler copy in-flight registers,
            // which waits for the loads.  Each slot is reloaded after its task
            // ran, so old and new descriptors share registers.
            for (int st0 = 0; st0 < Sp; st0 += RING) {
#pragma unroll
                for (int d = 0; d < RING; ++d) {
                    const int st = st0 + d;
                    if (tid < m.y) st_exec<PACKED>(v, ring[d]);
                    // the next steps' metadata after the task: its latency overlaps the barrier
                    const int2 m1 = sm[st + 1];
                    const int2 ma = sm[st + RING];
                    ring[d] = st_desc(drs, ma, tid);
                    __syncthreads();
                    m = m1;
                }
            }
            // first zero or non-finite pivot in elimination order (the values before it are exact)
            for (int j = tid; j < n; j += T)
                if (bad_pivot(v[j])) atomicMin(&s_bad, j + 1);
            __syncthreads();
            const int bad = s_bad == INT_MAX ? 0 : s_bad;
            if (!LIST && a.per_jacobian) {
                const double c = s_c[kk];
                double* xk = a.xk_too ? a.Xk + ((int64_t)s * es.K + kk) * n : nullptr;
                for (int q = tid; q < n; q += T) {
                    const double xq = bad ? __builtin_nan("") : y[q];
                    cx[q] = fmad(c, xq, kk == 0 ? 0.0 : cx[q]);
                    if (xk) xk[ix.perm[q]] = xq;
                }
            } else {
                double* xk = a.Xk + ((int64_t)s * es.K + kk) * n;
                for (int q = tid; q < n; q += T) xk[ix.perm[q]] = bad ? __builtin_nan("") : y[q];
            }
            if (tid == 0) a.info[s * es.K + kk] = bad;
            __syncthreads();
        }
        if (!LIST && a.per_jacobian)
            for (int q = tid; q < n; q += T) a.X[(int64_t)s * n + ix.perm[q]] = cx[q];
    }
}

}  // namespace

// Whether a schedule may fit (it is built, packed if need be, by steps_image;
// steps_ready tells whether it did).
bool steps_fit(const Symbolic& s, int32_t nrhs) { return nrhs == 1 && st_lds_doubles(s) < 0x7FFF; }

bool steps_ready(const SparseDevice& d) { return d.st.nsteps > 0; }

void steps_image(const Symbolic& s, const std::vector<int32_t>& r_pos, PlanImage& img, SparseDevice& d) {
    d.st = StepIdx{};
    if (!steps_fit(s, 1)) return;
    std::vector<int32_t> meta, desc, slot_l, slot_u;
    int32_t S = 0, pool = 0;
    // Unpacked when it fits two workgroups per CU (or packing cannot reach that); packed when
    // packing is what lets two workgroups share a CU, or the only way to fit at all.
    bool packed = false;
    const bool plain = build_schedule(s, r_pos, kStThreads, meta, desc, S, false, slot_l, slot_u, pool);
    if (!plain || st_lds_total(s.n, pool, S) > kStLdsPair) {
        std::vector<int32_t> pm, pd, pl, pu;
        int32_t pS = 0, pp = 0;
        if (build_schedule(s, r_pos, kStThreads, pm, pd, pS, true, pl, pu, pp) &&
            (!plain || st_lds_total(s.n, pp, pS) <= kStLdsPair)) {
            meta.swap(pm); desc.swap(pd); slot_l.swap(pl); slot_u.swap(pu);
            S = pS; pool = pp; packed = true;
        } else if (!plain) {
            return;
        }
    }
    if (S < 1 || desc.size() / 4 * 16 > (size_t)INT32_MAX) return;
    d.st.nsteps = S;
    d.st.threads = kStThreads;
    d.st.ndesc = (int32_t)(desc.size() / 4);
    img.bind(&d.st.meta, img.put(meta));
    img.bind(&d.st.desc, img.put(desc));
    img.bind(&d.st.slot_l, img.put(slot_l));
    img.bind(&d.st.slot_u, img.put(slot_u));
    d.st.pool = pool;
    d.st.packed = packed ? 1 : 0;
}

int64_t steps_lds_bytes(const SparseDevice& d) {
    return steps_ready(d) ? st_lds_total(d.idx.n, d.st.pool, d.st.nsteps) : 0;
}

int steps_per_cu(const SparseDevice& d) {
    return st_lds_total(d.idx.n, d.st.pool, d.st.nsteps) <= kStLdsPair ? 2 : 1;
}

// Once per process: the dynamic LDS limit of both kernel instances, and a check that
// the compiled static LDS stays within the headroom the schedule sizes assume.
hipError_t steps_kernel_attrs() {
    static hipError_t e = [] {
        const void* ks[6] = {(const void*)steps_kernel<kStThreads, true, false, kStAhead>,
                             (const void*)steps_kernel<kStThreads, false, false, kStAhead>,
                             (const void*)steps_kernel<kStThreads, true, false, kStRingShort>,
                             (const void*)steps_kernel<kStThreads, false, false, kStRingShort>,
                             (const void*)steps_kernel<kStThreads, true, true, kStAhead>,
                             (const void*)steps_kernel<kStThreads, false, true, kStAhead>};
        for (const void* k : ks) {
            hipFuncAttributes fa{};
            hipError_t r = hipFuncGetAttributes(&fa, k);
            if (r != hipSuccess) return r;
            if ((int64_t)fa.sharedSizeBytes > kStStaticLds) return hipErrorInvalidKernelFile;
            r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kStLdsMax);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }();
    return e;
}

hipError_t steps_run(const SparseDevice& d, int32_t nnz, int32_t batch, const double* values, const EpsSet& es,
                     const double* dvec, const double* B, double* X, double* Xk, int32_t* info, bool per_jacobian,
                     hipStream_t st, bool xk_too, const Knobs& kn) {
    if (!steps_ready(d) || d.st.threads != kStThreads) return hipErrorInvalidValue;
    StArgs a{};
    a.xk_too = per_jacobian && xk_too ? 1 : 0;
    a.sx = d.st;
    a.ix = d.idx;
    a.nnz = nnz; a.batch = batch; a.K = es.K; a.per_jacobian = per_jacobian ? 1 : 0;
    a.values = values; a.dvec = dvec; a.B = B; a.X = X; a.Xk = Xk; a.info = info;
    const int lds = (int)st_lds_total(d.idx.n, d.st.pool, d.st.nsteps);
    hipError_t e = steps_kernel_attrs();
    if (e != hipSuccess) return e;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int resident = cus * (kn.steps_wgcu == 1 ? 1 : steps_per_cu(d));
    const int64_t jobs = per_jacobian ? batch : (int64_t)batch * es.K;
    const int grid = (int)std::min<int64_t>(jobs, resident);
    const bool shortr = kn.ring == kStRingShort;
    if (d.st.packed && shortr)
        hipLaunchKernelGGL((steps_kernel<kStThreads, true, false, kStRingShort>), dim3(grid), dim3(kStThreads), lds, st, a, es);
    else if (d.st.packed)
        hipLaunchKernelGGL((steps_kernel<kStThreads, true, false, kStAhead>), dim3(grid), dim3(kStThreads), lds, st, a, es);
    else if (shortr)
        hipLaunchKernelGGL((steps_kernel<kStThreads, false, false, kStRingShort>), dim3(grid), dim3(kStThreads), lds, st, a, es);
    else
        hipLaunchKernelGGL((steps_kernel<kStThreads, false, false, kStAhead>), dim3(grid), dim3(kStThreads), lds, st, a, es);
    return hipGetLastError();
}

hipError_t steps_run_list(const SparseDevice& d, int32_t nnz, int32_t batch, const double* values, const EpsSet& es,
                          const double* dvec, const double* B, double* Xk, int32_t* info, const int32_t* list,
                          const int32_t* count, const double* scale, hipStream_t st) {
    if (!steps_ready(d) || d.st.threads != kStThreads) return hipErrorInvalidValue;
    StArgs a{};
    a.sx = d.st;
    a.ix = d.idx;
    a.nnz = nnz; a.batch = batch; a.K = es.K; a.per_jacobian = 0;
    a.values = values; a.dvec = dvec; a.B = B; a.X = nullptr; a.Xk = Xk; a.info = info;
    a.list = list; a.count = count; a.scale = scale;
    const int lds = (int)st_lds_total(d.idx.n, d.st.pool, d.st.nsteps);
    hipError_t e = steps_kernel_attrs();
    if (e != hipSuccess) return e;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the job count is on the device: every resident slot, idle ones leave at once
    const int grid = (int)std::min<int64_t>((int64_t)batch * es.K, (int64_t)cus * steps_per_cu(d));
    if (d.st.packed)
        hipLaunchKernelGGL((steps_kernel<kStThreads, true, true, kStAhead>), dim3(grid), dim3(kStThreads), lds, st, a, es);
    else
        hipLaunchKernelGGL((steps_kernel<kStThreads, false, true, kStAhead>), dim3(grid), dim3(kStThreads), lds, st, a, es);
    return hipGetLastError();
}

bool steps_per_jacobian(const SparseDevice& d, int32_t batch) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return batch >= cus * steps_per_cu(d);
}

hipError_t steps_solve(const SparseDevice& d, int32_t n, int32_t nnz, int32_t batch, const double* values,
                       const EpsSet& es, const double* dvec, const double* B, double* X, int32_t* info, double* Xk,
                       hipStream_t st, const Knobs& kn) {
    if (!steps_ready(d)) return hipErrorInvalidValue;
    // enough Jacobians to fill every resident workgroup slot: one workgroup per Jacobian,
    // combine fused; fewer: one workgroup per perturbed system and a combine launch
    const bool per_jacobian = kn.steps_mode < 0 ? steps_per_jacobian(d, batch) : kn.steps_mode == 1;
    hipError_t e = steps_run(d, nnz, batch, values, es, dvec, B, X, Xk, info, per_jacobian, st, false, kn);
    if (e != hipSuccess || per_jacobian) return e;
    return launch_combine((int64_t)n, batch, es, Xk, X, st);
}

}  // namespace psp
