// C-ABI of libdpsnn (declared in include/dpsnn.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <vector>

#include "dpsnn_internal.h"

namespace dpsnn {
std::vector<int64_t> fix_table(const dpsnn_params& p, const HostTables& T, int q, int b);
}

using namespace dpsnn;

namespace {

dpsnn_alloc_fn g_alloc = nullptr;
dpsnn_free_fn g_free = nullptr;
void* g_ctx = nullptr;

#define HIP_OK(expr)                          \
  do {                                        \
    if ((expr) != hipSuccess) return DPSNN_E_DEVICE; \
  } while (0)

void* dev_alloc(dpsnn_net* n, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (n->free_fn) {
    p = g_alloc ? g_alloc(bytes, n->alloc_ctx) : nullptr;
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    n->blocks.push_back(p);
    n->bytes_total += (int64_t)bytes;
  }
  return p;
}

void release_all(dpsnn_net* n) {
  for (void* p : n->blocks) {
    if (n->free_fn)
      n->free_fn(p, n->alloc_ctx);
    else
      (void)hipFree(p);
  }
  n->blocks.clear();
}

int acc_bytes(const dpsnn_params& p) { return p.acc_bits == 32 ? 4 : 8; }
int w_bytes(const dpsnn_params& p) {
  return p.weight_dtype == DPSNN_W_F32 ? 4 : p.weight_dtype == DPSNN_W_F16 ? 2 : 1;
}

// Parameters shared by every network of a batch (the step kernels use one
// value for all of them).
bool same_structure(const dpsnn_params& a, const dpsnn_params& b) {
  return a.K_out == b.K_out && a.d_min == b.d_min && a.d_max == b.d_max &&
         a.weight_dtype == b.weight_dtype && a.acc_bits == b.acc_bits &&
         a.q_frac_bits == b.q_frac_bits && a.rate_bin_steps == b.rate_bin_steps &&
         a.dt_ms == b.dt_ms && a.plastic == b.plastic &&
         (!a.plastic || (a.stdp_update_steps == b.stdp_update_steps &&
                         a.stdp_A_plus == b.stdp_A_plus && a.stdp_A_minus == b.stdp_A_minus &&
                         a.stdp_tau_plus == b.stdp_tau_plus &&
                         a.stdp_tau_minus == b.stdp_tau_minus &&
                         a.stdp_tau_y == b.stdp_tau_y && a.stdp_eta == b.stdp_eta &&
                         a.stdp_w_max == b.stdp_w_max));
}

int build_impl(dpsnn_net* n) {
  const int nn = (int)n->p.size();
  const dpsnn_params& p0 = n->p[0];
  n->T.resize(nn);
  for (int k = 0; k < nn; ++k) {
    const int rc = compute_tables(n->p[k], n->T[k]);
    if (rc != DPSNN_OK) return rc;
    if (!same_structure(p0, n->p[k]) || n->T[k].P != n->T[0].P) return DPSNN_E_INVAL;
  }
  const int P = n->T[0].P;
  HIP_OK(hipGetDevice(&n->device));
  const hipStream_t st = n->stream;
  const HostTables& T0 = n->T[0];
  // global index space: networks end to end, each padded to whole tiles
  n->base.resize(nn);
  n->mbase.resize(nn);
  int64_t gi = 0, gm = 0;
  for (int k = 0; k < nn; ++k) {
    n->base[k] = gi;
    n->mbase[k] = gm;
    gi += n->T[k].N_pad;
    gm += n->T[k].M;
    n->N_total += n->T[k].N;
  }
  n->N_pad = gi;
  n->rate_first.assign(nn, 0);
  n->pend.assign(nn, {});
  n->N_index = n->base[nn - 1] + n->T[nn - 1].N;
  n->M_total = (int32_t)gm;
  if (n->N_pad > (int64_t)kTargetMask) return DPSNN_E_INVAL;
  const int64_t Np = n->N_pad, M = gm;
  const int ab = acc_bytes(p0), wb = w_bytes(p0);
  const int rs = T0.row_stride;

  // ---- device memory
  int32_t* tgt = (int32_t*)dev_alloc(n, (size_t)Np * rs * 4);
  void* w = dev_alloc(n, (size_t)Np * rs * wb);
  n->bytes_rows = Np * rs * (4 + wb);
  float* V = (float*)dev_alloc(n, (size_t)Np * 4);
  float* c = (float*)dev_alloc(n, (size_t)Np * 4);
  uint8_t* ref = (uint8_t*)dev_alloc(n, (size_t)Np);
  void* slots = dev_alloc(n, (size_t)T0.D * Np * ab);
  n->bytes_state = Np * 9 + (int64_t)T0.D * Np * ab;
  const int64_t n_tiles = Np / 1024;
  // appended lists: list g takes the runs g, g + kSpkLists, ... of
  // 2^kSpkListShift consecutive tiles, and room for every neuron of them
  const int64_t tile_runs = (n_tiles + (1 << kSpkListShift) - 1) >> kSpkListShift;
  const int64_t spk_cap =
      (tile_runs + kSpkLists - 1) / kSpkLists * ((int64_t)1024 << kSpkListShift);
  int32_t* spk = (int32_t*)dev_alloc(n, (size_t)(kSpkLists * spk_cap) * 4);
  int32_t* blk_cnt = (int32_t*)dev_alloc(n, (size_t)n_tiles * 4);
  int32_t* tile_net = (int32_t*)dev_alloc(n, (size_t)n_tiles * 4);
  NetDev* nets = (NetDev*)dev_alloc(n, sizeof(NetDev) * nn);
  int2* log = (int2*)dev_alloc(n, (size_t)std::max<int64_t>(p0.spike_log_cap, 1) * 8);
  unsigned char* ctl = (unsigned char*)dev_alloc(n, 256 + 2 * kSpkLists * kSpkStride * 4);
  unsigned int* rates = (unsigned int*)dev_alloc(n, (size_t)p0.rate_bins_cap * M * P * 4);
  int64_t* sfix = (int64_t*)dev_alloc(n, (size_t)M * P * 8);
  if (!tgt || !w || !V || !c || !ref || !slots || !spk || !blk_cnt || !tile_net ||
      !nets || !log || !ctl || !rates || !sfix)
    return DPSNN_E_NOMEM;
  HIP_OK(hipMemsetAsync(slots, 0, (size_t)T0.D * Np * ab, st));
  HIP_OK(hipMemsetAsync(ctl, 0, 256 + 2 * kSpkLists * kSpkStride * 4, st));
  HIP_OK(hipMemsetAsync(blk_cnt, 0, (size_t)n_tiles * 4, st));
  HIP_OK(hipMemsetAsync(rates, 0, (size_t)p0.rate_bins_cap * M * P * 4, st));

  // int32 input slots: check at build that no step can leave the range.
  // The per-step sum at a neuron is bounded by the sum of |fixed-point
  // efficacy| over its incoming synapses plus the largest external sum.
  unsigned long long* absum = nullptr;
  int64_t ext_bound = 0;
  int64_t max_fix = 0;  // largest |fixed-point efficacy| of every table
  if (p0.acc_bits == 32 && p0.K_out > 0) {
    absum = (unsigned long long*)dev_alloc(n, (size_t)Np * 8 + 256);
    if (!absum) return DPSNN_E_NOMEM;
    HIP_OK(hipMemsetAsync(absum, 0, (size_t)Np * 8 + 256, st));
  }

  void* jx_all = dev_alloc(n, (size_t)nn * kMaxPops * kQuantN * ab);
  if (!jx_all) return DPSNN_E_NOMEM;
  std::vector<NetDev> nd(nn);
  bool all_two = P > 2;  // two classes of Eq. 2 constants in every network
  std::vector<int32_t> tn((size_t)n_tiles);
  std::vector<int64_t> sf((size_t)M * P);
  for (int k = 0; k < nn; ++k) {
    const dpsnn_params& p = n->p[k];
    const HostTables& T = n->T[k];
    const int64_t b = n->base[k];
    const uint32_t key0 = (uint32_t)n->seed[k], key1 = (uint32_t)(n->seed[k] >> 32);
    ext_bound = std::max(ext_bound, T.ext_bound);
    // per-network tables
    uint32_t* off_thr = (uint32_t*)dev_alloc(n, std::max<size_t>(T.off_thr.size(), 1) * 4);
    int32_t* off_xy = (int32_t*)dev_alloc(n, std::max<size_t>(T.off_xy.size(), 2) * 4);
    if (!off_thr || !off_xy) return DPSNN_E_NOMEM;
    if (!T.off_thr.empty())
      HIP_OK(hipMemcpyAsync(off_thr, T.off_thr.data(), T.off_thr.size() * 4,
                            hipMemcpyHostToDevice, st));
    if (!T.off_xy.empty())
      HIP_OK(hipMemcpyAsync(off_xy, T.off_xy.data(), T.off_xy.size() * 4,
                            hipMemcpyHostToDevice, st));
    // efficacy tables by (source pop, block), in the stored format; their
    // fixed-point values for the range check
    void* wtab[kMaxPops][kMaxPops] = {};
    int64_t* wfix_dev[kMaxPops][kMaxPops] = {};
    std::vector<std::vector<int64_t>> wf;  // staging: kept until the sync below
    for (int q = 0; q < T.P; ++q)
      for (int bb = 0; bb < T.tables(q); ++bb) {
        wtab[q][bb] = dev_alloc(n, (size_t)kQuantN * wb);
        if (!wtab[q][bb]) return DPSNN_E_NOMEM;
        const void* src = p.weight_dtype == DPSNN_W_F32 ? (const void*)T.wt32[q][bb].data()
                          : p.weight_dtype == DPSNN_W_F16 ? (const void*)T.wt16[q][bb].data()
                                                          : (const void*)T.wq8[q][bb].data();
        HIP_OK(hipMemcpyAsync(wtab[q][bb], src, (size_t)kQuantN * wb, hipMemcpyHostToDevice, st));
        for (int64_t v : fix_table(p, T, q, bb)) max_fix = std::max<int64_t>(max_fix, v < 0 ? -v : v);
        if (absum) {
          wfix_dev[q][bb] = (int64_t*)dev_alloc(n, (size_t)kQuantN * 8);
          if (!wfix_dev[q][bb]) return DPSNN_E_NOMEM;
          wf.push_back(fix_table(p, T, q, bb));
          // a plastic efficacy moves within [0, w_max] after the first
          // update: bound it by the larger of its start and w_max
          const bool exc = p.n_pops == 0 ? q == 0 : p.pop_exc[q] != 0;
          if (p.plastic && exc) {
            const int64_t wm = (int64_t)llrint(ldexp(p.stdp_w_max, p.q_frac_bits));
            for (int64_t& v : wf.back()) v = std::max<int64_t>(v < 0 ? -v : v, wm);
          }
          HIP_OK(hipMemcpyAsync(wfix_dev[q][bb], wf.back().data(), (size_t)kQuantN * 8,
                                hipMemcpyHostToDevice, st));
        }
      }
    // external fixed-point efficacies by target pop
    void* jx = static_cast<unsigned char*>(jx_all) + (size_t)k * kMaxPops * kQuantN * ab;
    std::vector<unsigned char> jxh((size_t)kMaxPops * kQuantN * ab, 0);
    for (int q = 0; q < T.P; ++q)
      for (int i = 0; i < kQuantN; ++i) {
        const int64_t v = T.jxfix[q][i];
        if (ab == 4) {
          const int32_t v32 = (int32_t)v;
          memcpy(&jxh[((size_t)q * kQuantN + i) * 4], &v32, 4);
        } else {
          memcpy(&jxh[((size_t)q * kQuantN + i) * 8], &v, 8);
        }
      }
    HIP_OK(hipMemcpyAsync(jx, jxh.data(), jxh.size(), hipMemcpyHostToDevice, st));
    // int8 scale per (module, source pop); modules of one network share the
    // parameters, hence the scale of their population
    for (int64_t m = 0; m < T.M; ++m)
      for (int q = 0; q < P; ++q) sf[(size_t)P * (n->mbase[k] + m) + q] = T.s8fix[q];
    for (int64_t tl = b / 1024; tl < (b + T.N_pad) / 1024; ++tl) tn[(size_t)tl] = k;

    InitArgs ia{};
    ia.N = T.N;
    ia.N_pad = T.N_pad;
    ia.K = p.K;
    ia.P = T.P;
    ia.key0 = key0;
    ia.key1 = key1;
    for (int q = 0; q < kMaxPops; ++q) {
      ia.pop_hi[q] = q < T.P - 1 ? T.pop_hi[q] : p.K;
      ia.E[q] = q < T.P ? (float)T.E[q] : 0.f;
      ia.Vth[q] = q < T.P ? (float)T.Vth[q] : 0.f;
    }
    ia.V = V + b;
    ia.c = c + b;
    ia.ref = ref + b;
    HIP_OK(launch_init(ia, st));

    GenArgs ga{};
    ga.N = T.N;
    ga.tgt_base = b;
    ga.K = p.K;
    ga.K_out = p.K_out;
    ga.row_stride = rs;
    ga.n_del = T.n_del;
    ga.d_min = p.d_min;
    ga.W = p.grid_w;
    ga.H = p.grid_h;
    ga.n_off = (int32_t)(T.off_xy.size() / 2);
    ga.open = T.open;
    ga.P = T.P;
    for (int q = 0; q < kMaxPops; ++q) {
      ga.pop_hi[q] = q < T.P - 1 ? T.pop_hi[q] : p.K;
      ga.n_blk[q] = q < T.P ? T.n_blk[q] : 0;
      int end = 0;
      for (int bb = 0; bb < kMaxPops; ++bb) {
        const bool on = q < T.P && bb < T.n_blk[q];
        end += on ? T.blk_n[q][bb] : 0;
        ga.blk_end[q][bb] = end;
        ga.blk_lo[q][bb] = on ? T.blk_lo[q][bb] : 0;
        ga.blk_hi[q][bb] = on ? T.blk_hi[q][bb] : 1;
        ga.blk_rule[q][bb] = on ? T.blk_rule[q][bb] : kRuleOwn;
        ga.wtab[q][bb] = wtab[q][bb];
        ga.wfix_tab[q][bb] = wfix_dev[q][bb];
      }
    }
    ga.key0 = key0;
    ga.key1 = key1;
    ga.off_thr = off_thr;
    ga.off_xy = off_xy;
    ga.tgt = tgt + b * rs;
    ga.w = static_cast<unsigned char*>(w) + (size_t)b * rs * wb;
    ga.absum = absum;
    if (p.K_out > 0) HIP_OK(launch_gen(ga, p.weight_dtype, st));
    HIP_OK(hipStreamSynchronize(st));

    NetDev& d = nd[k];
    memset(&d, 0, sizeof(d));
    d.base = b;
    d.N = T.N;
    d.mbase = (int32_t)n->mbase[k];
    d.K = p.K;
    d.P = T.P;
    d.key0 = key0;
    d.key1 = key1;
    for (int q = 0; q < kMaxPops; ++q) d.pop_hi[q] = q < T.P - 1 ? T.pop_hi[q] : p.K;
    {
      int sh = 0;
      while ((2ll << sh) <= p.K) ++sh;  // floor(log2 K)
      d.kshift = sh;
      d.kmag = (p.K & (p.K - 1)) == 0 ? 0u
                                      : (uint32_t)((((uint64_t)1 << (32 + sh)) / (uint64_t)p.K) + 1);
    }
    for (int q = 0; q < T.P; ++q) {
      d.Pm[q] = T.prop32[q][0];
      d.Pc[q] = T.prop32[q][1];
      d.PVc[q] = T.prop32[q][2];
      d.Iterm[q] = T.prop32[q][3];
      d.E[q] = (float)T.E[q];
      d.Vth[q] = (float)T.Vth[q];
      d.Vr[q] = (float)T.Vr[q];
      d.alpha[q] = (float)T.alpha[q];
      d.n_arp[q] = T.n_arp[q];
      d.n_pois[q] = T.n_pois[q];
      for (int x = 0; x < kMaxPois; ++x) d.pois[q][x] = T.pois[q][x];
      d.exc[q] = p.n_pops == 0 ? (q == 0) : (p.pop_exc[q] != 0);
    }
    // classes of equal Eq. 2 constants: a prefix of populations like
    // population 0 and the rest like the first population after it
    auto same = [&](int q, int r) {
      return memcmp(&d.Pm[q], &d.Pm[r], 4) == 0 && memcmp(&d.Pc[q], &d.Pc[r], 4) == 0 &&
             memcmp(&d.PVc[q], &d.PVc[r], 4) == 0 && memcmp(&d.Iterm[q], &d.Iterm[r], 4) == 0 &&
             memcmp(&d.E[q], &d.E[r], 4) == 0 && memcmp(&d.Vth[q], &d.Vth[r], 4) == 0 &&
             memcmp(&d.Vr[q], &d.Vr[r], 4) == 0 && memcmp(&d.alpha[q], &d.alpha[r], 4) == 0 &&
             d.n_arp[q] == d.n_arp[r];
    };
    int rep = 1;
    while (rep < T.P && same(rep, 0)) ++rep;
    bool two = true;
    for (int q = rep + 1; q < T.P; ++q) two = two && same(q, rep);
    d.cls_rep = rep < T.P ? rep : 0;
    d.cls_hi = rep < T.P ? d.pop_hi[rep - 1] : p.K;
    all_two = all_two && two;
  }
  HIP_OK(hipMemcpyAsync(nets, nd.data(), sizeof(NetDev) * nn, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(tile_net, tn.data(), tn.size() * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(sfix, sf.data(), sf.size() * 8, hipMemcpyHostToDevice, st));
  if (absum) {
    HIP_OK(launch_absum_max(absum, Np, absum + Np, st));
    unsigned long long mx = 0;
    HIP_OK(hipMemcpyAsync(&mx, absum + Np, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if ((double)mx + (double)ext_bound >= 2147483647.0) return DPSNN_E_RANGE;
  }
  HIP_OK(hipStreamSynchronize(st));

  // ---- step arguments
  StepArgs& a = n->sa;
  memset(&a, 0, sizeof(a));
  a.N_pad = Np;
  a.K_out = p0.K_out;
  a.row_stride = rs;
  a.D = T0.D;
  a.n_del = T0.n_del;
  a.d_min = p0.d_min;
  a.M = (int32_t)M;
  a.P = P;
  a.two_cls = all_two ? 1 : 0;
  a.n_tiles = (int32_t)n_tiles;
  a.deliver_blocks = (int32_t)std::min<int64_t>(1024, std::max<int64_t>(256, n_tiles));
  a.rate_bin_steps = p0.rate_bin_steps;
  a.rate_bins_cap = (int32_t)p0.rate_bins_cap;
  a.inv2q = ldexpf(1.0f, -p0.q_frac_bits);
  a.two_q = ldexpf(1.0f, p0.q_frac_bits);
  a.spike_log_cap = p0.spike_log_cap;
  a.nets = nets;
  a.tile_net = tile_net;
  a.jx = jx_all;
  a.V = V;
  a.c = c;
  a.ref = ref;
  a.slots = slots;
  a.tgt = tgt;
  a.w = w;
  a.sfix = sfix;
  a.spk = spk;
  a.spk_cap = spk_cap;
  a.blk_cnt = blk_cnt;
  a.spk_lists = 1;  // appended lists (merged reservations once queues exist);
                    // the autotuner also tries the other kinds
  a.log = log;
  a.log_base = reinterpret_cast<unsigned long long*>(ctl);
  a.n_spikes = reinterpret_cast<unsigned long long*>(ctl + 16);
  a.t_base = reinterpret_cast<uint32_t*>(ctl + 32);
  a.spk_n = reinterpret_cast<uint32_t*>(ctl + 256);  // spike-list counters
  a.rates = rates;
  n->ctl = ctl;

  // event queues: per tile an inbox for each step parity (2 x cap entries)
  // and one queue per slot (cap entries); none for more than 128 slots; the
  // default capacity shrinks so that the queues stay within 16 GiB
  int64_t qcap = p0.queue_cap == 0 ? kQueueDefaultCap
                 : p0.queue_cap < 0 ? 0 : p0.queue_cap;
  if (p0.K_out == 0 || T0.D > kQueueMaxSlots) qcap = 0;
  // binary16 and int8 efficacies travel as their stored codes (4-byte code
  // entries, whatever the slot width); binary32 ones in fixed point
  const int q_code = p0.weight_dtype == DPSNN_W_F16 ? kCodeF16
                     : p0.weight_dtype == DPSNN_W_I8 ? kCodeI8
                                                     : 0;
  const size_t eb = q_code      ? 4
                    : ab == 4   ? sizeof(QEntry<int32_t>)
                                : sizeof(QEntry<int64_t>);
  const int64_t per_cap = (int64_t)n_tiles * (T0.D + 4) * (int64_t)eb;  // bytes per unit of cap
  // int64 entries hold efficacies below 2^46 in fixed point (a plastic
  // efficacy up to w_max); past that, no queues
  const int64_t wmax_fix =
      p0.plastic ? (int64_t)llrint(ldexp(p0.stdp_w_max, p0.q_frac_bits)) : 0;
  if (!q_code && ab == 8 && (max_fix >= kQEntry64Max || wmax_fix >= kQEntry64Max)) qcap = 0;
  if (p0.queue_cap == 0 && qcap > 0) {
    const int64_t budget = (int64_t)16 << 30;
    qcap = std::min(qcap, budget / std::max<int64_t>(per_cap, 1));
    if (qcap < 64) qcap = 0;
  }
  // inbox entries are addressed with 32-bit indices: [2][tiles][2 cap]
  if (qcap > 0 && (int64_t)4 * n_tiles * qcap >= 0xFFFFFFFFll) return DPSNN_E_INVAL;
  if (qcap > 0) {
    a.q_cap = (int32_t)qcap;
    a.in_cap = (int32_t)(2 * qcap);
    a.route_blocks = (int32_t)std::min<int64_t>(n_tiles, 4096);
    const size_t n_in = (size_t)2 * n_tiles * a.in_cap;
    const size_t n_q = (size_t)n_tiles * T0.D * qcap;
    a.in_cnt = (uint32_t*)dev_alloc(n, (size_t)2 * n_tiles * kInboxStride * 4);
    a.in_q = dev_alloc(n, n_in * eb);
    a.q_cnt = (uint32_t*)dev_alloc(n, (size_t)n_tiles * T0.D * 4);
    a.q_q = dev_alloc(n, n_q * eb);
    a.s_dirty = (uint32_t*)dev_alloc(n, (size_t)n_tiles * T0.D * 4);
    if (!a.in_cnt || !a.in_q || !a.q_cnt || !a.q_q || !a.s_dirty) return DPSNN_E_NOMEM;
    HIP_OK(hipMemsetAsync(a.in_cnt, 0, (size_t)2 * n_tiles * kInboxStride * 4, st));
    HIP_OK(hipMemsetAsync(a.q_cnt, 0, (size_t)n_tiles * T0.D * 4, st));
    HIP_OK(hipMemsetAsync(a.s_dirty, 0, (size_t)n_tiles * T0.D * 4, st));
    HIP_OK(hipStreamSynchronize(st));
    // 4-byte queue entries when every efficacy (and a plastic one's
    // largest value) fits 21 bits
    a.q_packed = ab == 4 && max_fix < (1 << 21) && wmax_fix < (1 << 21);
    a.q_code = q_code;
    a.spk_lists = 2;  // appended lists, reservations merged per delivery block
    n->bytes_state += (int64_t)((n_in + n_q) * eb) +
                      (2 * n_tiles * kInboxStride + 2 * n_tiles * T0.D) * 4;
  }
  n->sched = n->N_total >= 65536 ? DPSNN_SCHED_SPLIT : DPSNN_SCHED_FUSED;

  // plasticity: per-synapse activation step and signal, per-neuron last
  // spike, the three binary32 tables; the split schedule only (a delivery
  // reads the targets' spike steps of the same step)
  if (p0.plastic) {
    n->sched = DPSNN_SCHED_SPLIT;
    const int32_t L = p0.stdp_update_steps;
    a.plastic = 1;
    a.stdp_L = L;
    a.stdp_eta = (float)p0.stdp_eta;
    a.stdp_wmax = (float)p0.stdp_w_max;
    a.syn_t = (int32_t*)dev_alloc(n, (size_t)Np * rs * 4);
    a.syn_y = (float*)dev_alloc(n, (size_t)Np * rs * 4);
    a.t_post = (int32_t*)dev_alloc(n, (size_t)Np * 4);
    float* tab = (float*)dev_alloc(n, (size_t)3 * L * 4);
    if (!a.syn_t || !a.syn_y || !a.t_post || !tab) return DPSNN_E_NOMEM;
    std::vector<float> h((size_t)3 * L);
    for (int32_t k = 0; k < L; ++k) {
      const double x = (double)k * p0.dt_ms;
      h[k] = (float)(p0.stdp_A_plus * exp(-x / p0.stdp_tau_plus));
      h[(size_t)L + k] = (float)(p0.stdp_A_minus * exp(-x / p0.stdp_tau_minus));
      h[(size_t)2 * L + k] = (float)exp(-x / p0.stdp_tau_y);
    }
    HIP_OK(hipMemcpyAsync(tab, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    a.stdp_tab = tab;
    HIP_OK(hipMemsetAsync(a.syn_t, 0xFF, (size_t)Np * rs * 4, st));  // -1: never
    HIP_OK(hipMemsetAsync(a.syn_y, 0, (size_t)Np * rs * 4, st));
    HIP_OK(hipMemsetAsync(a.t_post, 0xFF, (size_t)Np * 4, st));
    HIP_OK(hipStreamSynchronize(st));
    n->bytes_state += (int64_t)Np * rs * 8 + Np * 4;
  }
  return DPSNN_OK;
}

int build_common(const dpsnn_params* p, const uint64_t* seeds, int32_t n_nets,
                 dpsnn_net** out) {
  if (!p || !seeds || !out || n_nets < 1) return DPSNN_E_INVAL;
  *out = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<dpsnn_net> n(new dpsnn_net());
  n->p.assign(p, p + n_nets);
  n->seed.assign(seeds, seeds + n_nets);
  n->free_fn = g_free;
  n->alloc_ctx = g_ctx;
  const int rc = build_impl(n.get());
  if (rc != DPSNN_OK) {
    // parameter and range errors come before any device call
    if (!n->blocks.empty()) {
      (void)hipStreamSynchronize(n->stream);
      release_all(n.get());
    }
    return rc;
  }
  n->build_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = n.release();
  return DPSNN_OK;
}

}  // namespace

namespace {

// Device scratch of one analysis call: from the handle's allocator when it
// has one, else hipMalloc, freed when the call returns; or carved out of a
// fixed device buffer (arena), with no allocation at all; or only counted
// (measure: the pointers returned are placeholders and never used).
struct Scratch {
  dpsnn_free_fn free_fn = nullptr;
  void* ctx = nullptr;
  unsigned char* arena = nullptr;
  size_t arena_cap = 0;
  size_t used = 0;
  bool measure = false;
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    if (bytes == 0) bytes = 256;
    if (measure) {
      used += bytes;
      return reinterpret_cast<void*>((uintptr_t)used);
    }
    if (arena) {
      if (used + bytes > arena_cap) return nullptr;
      void* p = arena + used;
      used += bytes;
      return p;
    }
    void* p = nullptr;
    if (free_fn) {
      p = g_alloc ? g_alloc(bytes, ctx) : nullptr;
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    if (p) ptrs.push_back(p);
    return p;
  }
  ~Scratch() {
    for (void* p : ptrs) {
      if (free_fn)
        free_fn(p, ctx);
      else
        (void)hipFree(p);
    }
  }
};

// Checks of the analysis request shared by every entry point.
int waves_check(const WaveArgs& src, int32_t bin_steps, double dt_ms,
                const dpsnn_wave_params* wp, const dpsnn_wave_result* out, int64_t cap_tr,
                int64_t cap_w) {
  if (!wp || !out || wp->abi_version != DPSNN_ABI_VERSION || cap_tr < 0 || cap_w < 0)
    return DPSNN_E_INVAL;
  if (src.nb < 1 || src.nb > kWaveMaxBins || src.M < 1 || src.M > kWaveMaxModules ||
      src.P < 1 || wp->min_down < 1 || wp->min_up < 1 || wp->min_modules < 0 ||
      !(wp->noise_var >= 0.0) || !std::isfinite(wp->noise_var) || bin_steps < 1 ||
      !(dt_ms > 0.0))
    return DPSNN_E_INVAL;
  return DPSNN_OK;
}

// The scratch buffers of one analysis: every one is taken here, before any
// device work, except the log table when lnt_cap = 0 (then it is sized from
// the largest count once that is known).
struct WaveBufs {
  uint32_t* maxc;
  double* d_mean;
  double* d_z;
  double* d_lnt;
};
int waves_take(WaveArgs& a, const dpsnn_wave_params* wp, int64_t lnt_cap, Scratch& S,
               WaveBufs& B) {
  a.min_down = wp->min_down;
  a.min_up = wp->min_up;
  a.min_modules = wp->min_modules;
  a.cap_pm = a.nb / (a.min_down + a.min_up) + 1;
  const int64_t nt = (int64_t)a.M * a.cap_pm;
  B.maxc = (uint32_t*)S.get(4);
  a.cnt = (uint32_t*)S.get((size_t)a.M * 4);
  a.tr_k = (uint32_t*)S.get((size_t)nt * 4);
  a.tr_q = (uint32_t*)S.get((size_t)nt * 4);
  a.tr_T = (double*)S.get((size_t)nt * 8);
  a.hist = (uint32_t*)S.get((size_t)a.nb * 4);
  a.fill = (uint32_t*)S.get((size_t)a.nb * 4);
  a.off = (uint32_t*)S.get((size_t)(a.nb + 1) * 4);
  a.keys = (unsigned long long*)S.get((size_t)nt * 8);
  a.pos = (uint32_t*)S.get((size_t)nt * 4);
  a.nxt = (uint32_t*)S.get((size_t)nt * 4);
  a.out_module = (int32_t*)S.get((size_t)nt * 4);
  a.out_T = (double*)S.get((size_t)nt * 8);
  a.out_wave = (int32_t*)S.get((size_t)nt * 4);
  a.wave_first = (int32_t*)S.get((size_t)(nt + 1) * 4);
  a.n_waves = (int32_t*)S.get(4);
  a.wave_speed = (double*)S.get((size_t)nt * 8);
  a.wave_t0 = (double*)S.get((size_t)nt * 8);
  a.wave_n = (int32_t*)S.get((size_t)nt * 4);
  a.grid = (double*)S.get((size_t)kWaveBatch * a.M * 8);
  B.d_mean = (double*)S.get(8);
  B.d_z = (double*)S.get((size_t)kQuantN * 8);
  B.d_lnt = lnt_cap > 0 ? (double*)S.get((size_t)lnt_cap * 8) : nullptr;
  for (const void* q : {(const void*)B.maxc, (const void*)a.cnt, (const void*)a.tr_k,
                        (const void*)a.tr_q, (const void*)a.tr_T, (const void*)a.hist,
                        (const void*)a.fill, (const void*)a.off, (const void*)a.keys,
                        (const void*)a.pos, (const void*)a.nxt,
                        (const void*)a.out_module, (const void*)a.out_T,
                        (const void*)a.out_wave, (const void*)a.wave_first,
                        (const void*)a.n_waves, (const void*)a.wave_speed,
                        (const void*)a.wave_t0, (const void*)a.wave_n, (const void*)a.grid,
                        (const void*)B.d_mean, (const void*)B.d_z})
    if (!q) return DPSNN_E_NOMEM;
  if (lnt_cap > 0 && !B.d_lnt) return DPSNN_E_NOMEM;
  return DPSNN_OK;
}

// The slow-wave analysis over a window of count bins (see dpsnn.h).
// lnt_host / lnt_cap: a host table of log(i), i < lnt_cap, whose device copy
// is taken from S up front (no allocation once the count is known); null:
// the table is built and its buffer taken after the largest count is read.
int waves_impl(const WaveArgs& src, int32_t bin_steps, double dt_ms,
               const dpsnn_wave_params* wp, hipStream_t st, Scratch& S,
               const double* lnt_host, int64_t lnt_cap,
               dpsnn_wave_result* out, int32_t* h_mod, double* h_T, int32_t* h_wave,
               int64_t cap_tr, double* h_speed, double* h_t0, int32_t* h_n, int64_t cap_w) {
  int rc = waves_check(src, bin_steps, dt_ms, wp, out, cap_tr, cap_w);
  if (rc != DPSNN_OK) return rc;
  WaveArgs a = src;
  a.dbin = (double)bin_steps * dt_ms;
  a.sd = sqrt(wp->noise_var);
  a.key0 = (uint32_t)wp->seed;
  a.key1 = (uint32_t)(wp->seed >> 32);
  WaveBufs B{};
  rc = waves_take(a, wp, lnt_host ? lnt_cap : 0, S, B);
  if (rc != DPSNN_OK) return rc;
  uint32_t* maxc = B.maxc;
  double* d_mean = B.d_mean;
  a.z = B.d_z;
  const std::vector<double>& z = standard_normal_grid();
  HIP_OK(hipMemcpyAsync(B.d_z, z.data(), (size_t)kQuantN * 8, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemsetAsync(maxc, 0, 4, st));
  HIP_OK(hipMemsetAsync(a.hist, 0, (size_t)a.nb * 4, st));
  HIP_OK(hipMemsetAsync(a.fill, 0, (size_t)a.nb * 4, st));
  HIP_OK(hipMemsetAsync(a.n_waves, 0, 4, st));
  HIP_OK(launch_wave_max(a, maxc, st));
  uint32_t mx = 0;
  HIP_OK(hipMemcpyAsync(&mx, maxc, 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  // log(i) for every count + 1 that can occur (host binary64 log)
  if (lnt_host) {
    if ((int64_t)mx + 2 > lnt_cap) return DPSNN_E_SCRATCH;
    a.lnt = B.d_lnt;
    HIP_OK(hipMemcpyAsync(B.d_lnt, lnt_host, ((size_t)mx + 2) * 8, hipMemcpyHostToDevice, st));
  } else {
    std::vector<double> lnt((size_t)mx + 2);
    lnt[0] = -INFINITY;
    for (size_t i = 1; i < lnt.size(); ++i) lnt[i] = log((double)i);
    double* d_lnt = (double*)S.get(lnt.size() * 8);
    if (!d_lnt) return DPSNN_E_NOMEM;
    a.lnt = d_lnt;
    HIP_OK(hipMemcpyAsync(d_lnt, lnt.data(), lnt.size() * 8, hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));  // lnt is released on return
  }
  HIP_OK(launch_wave_transitions(a, st));
  int32_t nw = 0;
  uint32_t total = 0;
  HIP_OK(hipMemcpyAsync(&nw, a.n_waves, 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(&total, a.off + a.nb, 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int32_t w0 = 0; w0 < nw; w0 += kWaveBatch)
    HIP_OK(launch_wave_speed(a, w0, std::min<int32_t>(kWaveBatch, nw - w0), st));
  HIP_OK(launch_wave_mean(a, d_mean, st));
  double mean = 0.0;
  HIP_OK(hipMemcpyAsync(&mean, d_mean, 8, hipMemcpyDeviceToHost, st));
  const int64_t ntr = std::min<int64_t>(total, cap_tr);
  const int64_t nwc = std::min<int64_t>(nw, cap_w);
  if (ntr > 0) {
    if (h_mod) HIP_OK(hipMemcpyAsync(h_mod, a.out_module, ntr * 4, hipMemcpyDeviceToHost, st));
    if (h_T) HIP_OK(hipMemcpyAsync(h_T, a.out_T, ntr * 8, hipMemcpyDeviceToHost, st));
    if (h_wave) HIP_OK(hipMemcpyAsync(h_wave, a.out_wave, ntr * 4, hipMemcpyDeviceToHost, st));
  }
  if (nwc > 0) {
    if (h_speed) HIP_OK(hipMemcpyAsync(h_speed, a.wave_speed, nwc * 8, hipMemcpyDeviceToHost, st));
    if (h_t0) HIP_OK(hipMemcpyAsync(h_t0, a.wave_t0, nwc * 8, hipMemcpyDeviceToHost, st));
    if (h_n) HIP_OK(hipMemcpyAsync(h_n, a.wave_n, nwc * 4, hipMemcpyDeviceToHost, st));
  }
  HIP_OK(hipStreamSynchronize(st));
  out->bin0 = a.bin0;
  out->n_bins = a.nb;
  out->n_transitions = total;
  out->n_waves = nw;
  out->mean_speed = mean;
  return DPSNN_OK;
}

// ---- allocation-free slow-wave analysis -----------------------------------
// A fixed device buffer for dpsnn_waves_counts_static: every GPU the library
// runs on holds one copy until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and only that address is passed on.
constexpr size_t kWaveScratchBytes = (size_t)64 << 20;
constexpr int64_t kWaveScratchMaxCount = 65535;  // largest count per module and bin
static __device__ __align__(256) unsigned char scratch[kWaveScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::vector<double> g_lnt;  // log(i), i <= kWaveScratchMaxCount + 1, built once

// The scratch's device address on the current device, and the log table.
int scratch_setup(void** ptr, const double** lnt) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return DPSNN_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DPSNN_E_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  if (g_lnt.empty()) {
    g_lnt.resize((size_t)kWaveScratchMaxCount + 2);
    g_lnt[0] = -INFINITY;
    for (size_t i = 1; i < g_lnt.size(); ++i) g_lnt[i] = log((double)i);
    (void)standard_normal_grid();  // built once, used by every call
  }
  *ptr = g_scratch_ptr[dev];
  *lnt = g_lnt.data();
  return DPSNN_OK;
}

}  // namespace

extern "C" {

int dpsnn_set_allocator(dpsnn_alloc_fn alloc, dpsnn_free_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr)) return DPSNN_E_INVAL;
  g_alloc = alloc;
  g_free = release;
  g_ctx = ctx;
  return DPSNN_OK;
}

int dpsnn_build(const dpsnn_params* p, uint64_t seed, dpsnn_net** out) {
  return build_common(p, &seed, 1, out);
}

int dpsnn_build_batch(const dpsnn_params* p, const uint64_t* seeds, int32_t n_nets,
                      dpsnn_net** out) {
  return build_common(p, seeds, n_nets, out);
}

int dpsnn_net_info(dpsnn_net* n, int32_t k, int64_t* base, int64_t* n_neurons,
                   int64_t* module_base, int64_t* n_modules) {
  if (!n || k < 0 || k >= (int32_t)n->p.size()) return DPSNN_E_INVAL;
  if (base) *base = n->base[k];
  if (n_neurons) *n_neurons = n->T[k].N;
  if (module_base) *module_base = n->mbase[k];
  if (n_modules) *n_modules = n->T[k].M;
  return DPSNN_OK;
}

int dpsnn_set_stream(dpsnn_net* n, void* s) {
  if (!n) return DPSNN_E_INVAL;
  n->stream = (hipStream_t)s;
  return DPSNN_OK;
}

}  // extern "C"

namespace {

void drop_graph(dpsnn_net* n) {
  if (n->graph) (void)hipGraphExecDestroy(n->graph);
  n->graph = nullptr;
  n->graph_K = 0;
  n->graph_sched = -1;
  n->graph_stream = nullptr;
}

// First rate bin that some network of the handle has not drained.
int64_t rate_first_min(const dpsnn_net* n) {
  return *std::min_element(n->rate_first.begin(), n->rate_first.end());
}

// Capture graph_steps steps of the current schedule followed by the step
// counter update; replays then need no host work per step.
int ensure_graph(dpsnn_net* n) {
  if (n->graph && n->graph_sched == n->sched && n->graph_stream == n->stream &&
      n->graph_blocks == n->sa.deliver_blocks && n->graph_lists == n->sa.spk_lists &&
      n->graph_routes == n->sa.route_blocks && n->graph_K == n->graph_steps)
    return DPSNN_OK;
  drop_graph(n);
  hipGraph_t g = nullptr;
  HIP_OK(hipStreamBeginCapture(n->stream, hipStreamCaptureModeThreadLocal));
  bool ok = true;
  for (int64_t k = 0; k < n->graph_steps && ok; ++k)
    ok = launch_step(n->sa, n->p[0].weight_dtype, n->p[0].acc_bits, n->sched, (uint32_t)k,
                     n->stream) == hipSuccess;
  if (ok) ok = launch_tick(n->sa, (uint32_t)n->graph_steps, 0, n->stream) == hipSuccess;
  const hipError_t e = hipStreamEndCapture(n->stream, &g);
  if (!ok || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return DPSNN_E_DEVICE;
  }
  hipGraphExec_t ge = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return DPSNN_E_DEVICE;
  n->graph = ge;
  n->graph_K = (int)n->graph_steps;
  n->graph_sched = n->sched;
  n->graph_blocks = n->sa.deliver_blocks;
  n->graph_lists = n->sa.spk_lists;
  n->graph_routes = n->sa.route_blocks;
  n->graph_stream = n->stream;
  return DPSNN_OK;
}

}  // namespace

extern "C" {

int dpsnn_set_schedule(dpsnn_net* n, int32_t sched) {
  if (!n || sched < DPSNN_SCHED_FUSED || sched > DPSNN_SCHED_PERSIST) return DPSNN_E_INVAL;
  if (sched != DPSNN_SCHED_SPLIT && n->sa.plastic) return DPSNN_E_INVAL;
  n->sched = sched;
  return DPSNN_OK;
}

int dpsnn_set_delivery(dpsnn_net* n, int32_t deliver_blocks, int32_t spike_lists) {
  if (!n || deliver_blocks < 0 || deliver_blocks > (1 << 20) || spike_lists < -1 ||
      spike_lists > 2 || (spike_lists == 0 && n->sa.n_tiles > kMaxScanTiles))
    return DPSNN_E_INVAL;
  if (deliver_blocks > 0) n->sa.deliver_blocks = deliver_blocks;
  if (spike_lists >= 0) n->sa.spk_lists = spike_lists;
  return DPSNN_OK;
}

int dpsnn_set_routing(dpsnn_net* n, int32_t route_blocks) {
  if (!n || route_blocks < 0 || route_blocks > n->sa.n_tiles) return DPSNN_E_INVAL;
  if (n->sa.q_cap == 0) return DPSNN_E_STATE;
  n->sa.route_blocks =
      route_blocks ? route_blocks : (int32_t)std::min<int64_t>(n->sa.n_tiles, 4096);
  return DPSNN_OK;
}

int dpsnn_set_graph_steps(dpsnn_net* n, int64_t steps) {
  if (!n || steps < 0 || steps > 100000) return DPSNN_E_INVAL;
  n->graph_steps = steps;
  return DPSNN_OK;
}

// n_steps steps: captured graphs for the bulk, the rest launched directly;
// the persistent schedule: launches of up to kPersistSteps steps.
constexpr int64_t kPersistSteps = 4096;
static int run_steps(dpsnn_net* n, int64_t n_steps) {
  if (n->sched == DPSNN_SCHED_PERSIST) {
    for (int64_t done = 0; done < n_steps;) {
      const int64_t k = std::min<int64_t>(n_steps - done, kPersistSteps);
      HIP_OK(launch_persist(n->sa, n->p[0].weight_dtype, n->p[0].acc_bits, 0, (uint32_t)k,
                            n->stream));
      HIP_OK(launch_tick(n->sa, (uint32_t)k, 0, n->stream));
      done += k;
    }
    n->t += n_steps;
    return DPSNN_OK;
  }
  int64_t done = 0;
  if (n->stream && n->graph_steps > 0 && n_steps >= n->graph_steps) {
    const int rc = ensure_graph(n);
    if (rc != DPSNN_OK) return rc;
    while (n_steps - done >= n->graph_K) {
      HIP_OK(hipGraphLaunch(n->graph, n->stream));
      done += n->graph_K;
    }
  }
  const int64_t rest = n_steps - done;
  if (rest > 0) {
    for (int64_t k = 0; k < rest; ++k)
      HIP_OK(launch_step(n->sa, n->p[0].weight_dtype, n->p[0].acc_bits, n->sched, (uint32_t)k,
                         n->stream));
    HIP_OK(launch_tick(n->sa, (uint32_t)rest, 0, n->stream));
  }
  n->t += n_steps;
  return DPSNN_OK;
}

int dpsnn_step(dpsnn_net* n, int64_t n_steps) {
  if (!n || n_steps < 0) return DPSNN_E_INVAL;
  if (n_steps == 0) return DPSNN_OK;
  if (n->t + n_steps > (n->sa.plastic ? 0x7FFFFFFFll : 0xFFFFFFFFll)) return DPSNN_E_INVAL;
  const int64_t last_bin = (n->t + n_steps - 1) / n->p[0].rate_bin_steps;
  if (last_bin - rate_first_min(n) + 1 > n->p[0].rate_bins_cap) return DPSNN_E_RATES_FULL;
  // the fused schedule advances both spike-log bases: align them after the
  // split or persistent schedule
  if (n->sched == DPSNN_SCHED_FUSED && n->last_sched >= 0 && n->last_sched != DPSNN_SCHED_FUSED)
    HIP_OK(launch_tick(n->sa, 0, 1, n->stream));
  n->last_sched = n->sched;
  if (!n->sa.plastic) return run_steps(n, n_steps);
  // plastic: steps up to each update time, then the efficacy update
  const int64_t U = n->sa.stdp_L;
  for (int64_t left = n_steps; left > 0;) {
    const int64_t k = std::min<int64_t>(left, U - n->t % U);
    const int rc = run_steps(n, k);
    if (rc != DPSNN_OK) return rc;
    left -= k;
    if (n->t % U == 0) HIP_OK(launch_stdp_update(n->sa, (int32_t)n->t, n->stream));
  }
  return DPSNN_OK;
}

int dpsnn_autotune(dpsnn_net* n, int64_t probe_steps, int32_t* chosen) {
  if (!n || probe_steps < 1) return DPSNN_E_INVAL;
  // candidates: the fused schedule, and the split one with several grids of
  // the delivery kernel, each with per-tile and with appended spike lists
  // (with and without merged reservations)
  struct Cand {
    int sched;
    int32_t blocks;
    int32_t lists;
  };
  std::vector<Cand> cands;
  if (!n->sa.plastic) {
    cands.push_back({DPSNN_SCHED_FUSED, n->sa.deliver_blocks, n->sa.spk_lists});
    cands.push_back({DPSNN_SCHED_PERSIST, n->sa.deliver_blocks, 1});
  }
  const int32_t tiles = n->sa.n_tiles;
  for (int32_t lists : {0, 1, 2}) {
    if (!lists && tiles > kMaxScanTiles) continue;
    if (lists == 2 && !n->sa.q_cap) continue;  // merged reservations need queues
    for (int32_t b : {std::min<int32_t>(1024, std::max<int32_t>(256, tiles)), 256, 512, 1024,
                      2048}) {
      bool seen = false;
      for (const Cand& c : cands)
        seen |= c.sched == DPSNN_SCHED_SPLIT && c.blocks == b && c.lists == lists;
      if (!seen) cands.push_back({DPSNN_SCHED_SPLIT, b, lists});
    }
  }
  // runs of K steps (whole graph replays when graphs are in use): one
  // untimed run per candidate, then `rounds` timed runs of every candidate
  // in turn, so that all of them see the same mix of activity
  const bool graphs = n->stream && n->graph_steps > 0;
  const int64_t K = graphs ? n->graph_steps : std::min<int64_t>(probe_steps, 128);
  const int64_t rounds = std::max<int64_t>(1, probe_steps / K);
  const size_t nc = cands.size();
  auto use = [&](const Cand& c) {
    n->sched = c.sched;
    n->sa.deliver_blocks = c.blocks;
    n->sa.spk_lists = c.lists;
  };
  Cand best{n->sched, n->sa.deliver_blocks, n->sa.spk_lists};
  std::vector<hipEvent_t> ev((size_t)2 * nc * rounds, nullptr);
  int rc = DPSNN_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) rc = DPSNN_E_DEVICE;
  for (size_t i = 0; i < nc && rc == DPSNN_OK; ++i) {
    use(cands[i]);
    rc = dpsnn_step(n, K);
  }
  for (int64_t r = 0; r < rounds && rc == DPSNN_OK; ++r) {
    for (size_t i = 0; i < nc && rc == DPSNN_OK; ++i) {
      use(cands[i]);
      // the graph is captured before the timed run (the persistent schedule
      // launches directly)
      if (graphs && n->sched != DPSNN_SCHED_PERSIST && (rc = ensure_graph(n)) != DPSNN_OK)
        break;
      hipEvent_t* e = &ev[(size_t)2 * (r * nc + i)];
      if (hipEventRecord(e[0], n->stream) != hipSuccess) { rc = DPSNN_E_DEVICE; break; }
      if ((rc = dpsnn_step(n, K)) != DPSNN_OK) break;
      if (hipEventRecord(e[1], n->stream) != hipSuccess) rc = DPSNN_E_DEVICE;
    }
  }
  if (rc == DPSNN_OK && hipStreamSynchronize(n->stream) != hipSuccess) rc = DPSNN_E_DEVICE;
  if (rc == DPSNN_OK) {
    double best_ms = -1.0;
    for (size_t i = 0; i < nc; ++i) {
      double sum = 0.0;
      for (int64_t r = 0; r < rounds; ++r) {
        const size_t k = (size_t)2 * (r * nc + i);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        sum += ms;
      }
      if (best_ms < 0.0 || sum < best_ms) {
        best_ms = sum;
        best = cands[i];
      }
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  use(best);
  if (chosen) *chosen = best.sched;
  return rc;
}

int dpsnn_profile_steps(dpsnn_net* n, int64_t n_steps, double* host_ms) {
  if (!n || n_steps < 1 || !host_ms) return DPSNN_E_INVAL;
  if (n->t + n_steps > (n->sa.plastic ? 0x7FFFFFFFll : 0xFFFFFFFFll)) return DPSNN_E_INVAL;
  const int64_t last_bin = (n->t + n_steps - 1) / n->p[0].rate_bin_steps;
  if (last_bin - rate_first_min(n) + 1 > n->p[0].rate_bins_cap) return DPSNN_E_RATES_FULL;
  if (n->sched == DPSNN_SCHED_FUSED && n->last_sched >= 0 && n->last_sched != DPSNN_SCHED_FUSED)
    HIP_OK(launch_tick(n->sa, 0, 1, n->stream));
  n->last_sched = n->sched;
  std::vector<hipEvent_t> ev((size_t)3 * n_steps);
  for (auto& e : ev) HIP_OK(hipEventCreate(&e));
  int rc = DPSNN_OK;
  for (int64_t k = 0; k < n_steps && rc == DPSNN_OK; ++k) {
    hipEvent_t* e = &ev[(size_t)3 * k];
    if (hipEventRecord(e[0], n->stream) != hipSuccess) rc = DPSNN_E_DEVICE;
    if (n->sched == DPSNN_SCHED_SPLIT) {
      if (launch_phase(n->sa, n->p[0].weight_dtype, n->p[0].acc_bits, 0, (uint32_t)k, n->stream) !=
              hipSuccess ||
          hipEventRecord(e[1], n->stream) != hipSuccess ||
          launch_phase(n->sa, n->p[0].weight_dtype, n->p[0].acc_bits, 1, (uint32_t)k, n->stream) !=
              hipSuccess)
        rc = DPSNN_E_DEVICE;
    } else {
      if (launch_step(n->sa, n->p[0].weight_dtype, n->p[0].acc_bits, n->sched, (uint32_t)k,
                      n->stream) != hipSuccess ||
          hipEventRecord(e[1], n->stream) != hipSuccess)
        rc = DPSNN_E_DEVICE;
    }
    if (hipEventRecord(e[2], n->stream) != hipSuccess) rc = DPSNN_E_DEVICE;
    const int64_t T = n->t + k + 1;  // plastic: the update after step T - 1
    if (n->sa.plastic && T % n->sa.stdp_L == 0 &&
        launch_stdp_update(n->sa, (int32_t)T, n->stream) != hipSuccess)
      rc = DPSNN_E_DEVICE;
  }
  if (rc == DPSNN_OK && launch_tick(n->sa, (uint32_t)n_steps, 0, n->stream) != hipSuccess)
    rc = DPSNN_E_DEVICE;
  if (rc == DPSNN_OK && hipStreamSynchronize(n->stream) != hipSuccess) rc = DPSNN_E_DEVICE;
  double t0 = 0.0, t1 = 0.0;
  for (int64_t k = 0; k < n_steps && rc == DPSNN_OK; ++k) {
    float a = 0.f, b = 0.f;
    (void)hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]);
    (void)hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]);
    t0 += a;
    t1 += b;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc != DPSNN_OK) return rc;
  n->t += n_steps;
  host_ms[0] = t0;
  host_ms[1] = t1;
  return DPSNN_OK;
}

static int log_count(dpsnn_net* n, unsigned long long* cnt) {
  HIP_OK(hipMemcpy(cnt, n->sa.log_base + (n->t & 1), 8, hipMemcpyDeviceToHost));
  return DPSNN_OK;
}

int dpsnn_sync(dpsnn_net* n) {
  if (!n) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  unsigned long long cnt = 0;
  const int rc = log_count(n, &cnt);
  if (rc != DPSNN_OK) return rc;
  if ((int64_t)cnt > n->p[0].spike_log_cap || n->log_overflow) return DPSNN_E_SPIKELOG_FULL;
  return DPSNN_OK;
}

// Move the device spike log into the per-network host lists and empty it.
static int drain_log(dpsnn_net* n) {
  HIP_OK(hipStreamSynchronize(n->stream));
  unsigned long long cnt = 0;
  const int rc = log_count(n, &cnt);
  if (rc != DPSNN_OK) return rc;
  if ((int64_t)cnt > n->p[0].spike_log_cap) n->log_overflow = true;
  const int64_t have = std::min<int64_t>((int64_t)cnt, n->p[0].spike_log_cap);
  if (have == 0) return DPSNN_OK;
  std::vector<int2> buf((size_t)have);
  HIP_OK(hipMemcpy(buf.data(), n->sa.log, (size_t)have * 8, hipMemcpyDeviceToHost));
  for (const int2& e : buf) {
    // network of a global id: the last base at or below it
    const size_t k =
        (size_t)(std::upper_bound(n->base.begin(), n->base.end(), (int64_t)e.y) -
                 n->base.begin()) - 1;
    n->pend[k].push_back(e);
  }
  HIP_OK(hipMemsetAsync(n->sa.log_base, 0, 16, n->stream));
  HIP_OK(hipStreamSynchronize(n->stream));
  return DPSNN_OK;
}

static bool by_step_id(const int2& a, const int2& b) {
  return a.x != b.x ? a.x < b.x : a.y < b.y;
}

// Hand out the pending spikes of networks [k0, k1), ids minus `off`.
static int hand_out(dpsnn_net* n, int32_t k0, int32_t k1, int64_t off, int32_t* host_step,
                    int32_t* host_id, int64_t cap, int64_t* n_out) {
  int64_t have = 0;
  for (int32_t k = k0; k < k1; ++k) have += (int64_t)n->pend[k].size();
  *n_out = have;
  if (cap < have || (have > 0 && (!host_step || !host_id))) return DPSNN_OK;
  std::vector<int2> buf;
  buf.reserve((size_t)have);
  for (int32_t k = k0; k < k1; ++k) {
    buf.insert(buf.end(), n->pend[k].begin(), n->pend[k].end());
    std::vector<int2>().swap(n->pend[k]);
  }
  std::sort(buf.begin(), buf.end(), by_step_id);
  for (int64_t i = 0; i < have; ++i) {
    host_step[i] = buf[(size_t)i].x;
    host_id[i] = (int32_t)(buf[(size_t)i].y - off);
  }
  const bool overflow = n->log_overflow;
  n->log_overflow = false;
  return overflow ? DPSNN_E_SPIKELOG_FULL : DPSNN_OK;
}

int dpsnn_read_spikes(dpsnn_net* n, int32_t* host_step, int32_t* host_id, int64_t cap,
                      int64_t* n_out) {
  if (!n || !n_out || cap < 0) return DPSNN_E_INVAL;
  const int rc = drain_log(n);
  if (rc != DPSNN_OK) return rc;
  return hand_out(n, 0, (int32_t)n->p.size(), 0, host_step, host_id, cap, n_out);
}

int dpsnn_read_spikes_net(dpsnn_net* n, int32_t k, int32_t* host_step, int32_t* host_id,
                          int64_t cap, int64_t* n_out) {
  if (!n || !n_out || cap < 0 || k < 0 || k >= (int32_t)n->p.size()) return DPSNN_E_INVAL;
  const int rc = drain_log(n);
  if (rc != DPSNN_OK) return rc;
  return hand_out(n, k, k + 1, n->base[k], host_step, host_id, cap, n_out);
}

// Copy (and clear on the device) the counts of modules [m0, m0 + nm) of
// bins [first, first + nb) of the rate ring into host [nb][nm][P]: at most
// two 2-D copies (the ring wraps once).
static int drain_bins(dpsnn_net* n, int64_t first, int64_t nb, int64_t m0, int64_t nm,
                      uint32_t* host) {
  const int64_t P = n->sa.P, per = (int64_t)n->M_total * P;
  const int64_t cap = n->p[0].rate_bins_cap;
  for (int64_t b = 0; b < nb;) {
    const int64_t src = (first + b) % cap;
    const int64_t run = std::min<int64_t>(nb - b, cap - src);
    unsigned int* d = n->sa.rates + src * per + m0 * P;
    HIP_OK(hipMemcpy2D(host + b * nm * P, (size_t)(nm * P * 4), d, (size_t)(per * 4),
                       (size_t)(nm * P * 4), (size_t)run, hipMemcpyDeviceToHost));
    HIP_OK(hipMemset2DAsync(d, (size_t)(per * 4), 0, (size_t)(nm * P * 4), (size_t)run,
                            n->stream));
    b += run;
  }
  HIP_OK(hipStreamSynchronize(n->stream));
  return DPSNN_OK;
}

int dpsnn_read_rates(dpsnn_net* n, uint32_t* host_counts, int64_t cap_bins, int64_t* n_bins) {
  if (!n || !n_bins || cap_bins < 0) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  const int64_t done = n->t / n->p[0].rate_bin_steps;
  const int64_t first = rate_first_min(n);
  const int64_t nb = done - first;
  *n_bins = nb;
  if (nb <= 0 || cap_bins < nb || !host_counts) return DPSNN_OK;
  const int rc = drain_bins(n, first, nb, 0, n->M_total, host_counts);
  if (rc != DPSNN_OK) return rc;
  std::fill(n->rate_first.begin(), n->rate_first.end(), done);
  return DPSNN_OK;
}

int dpsnn_read_rates_net(dpsnn_net* n, int32_t k, uint32_t* host_counts, int64_t cap_bins,
                         int64_t* n_bins) {
  if (!n || !n_bins || cap_bins < 0 || k < 0 || k >= (int32_t)n->p.size())
    return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  const int64_t done = n->t / n->p[0].rate_bin_steps;
  const int64_t nb = done - n->rate_first[k];
  *n_bins = nb;
  if (nb <= 0 || cap_bins < nb || !host_counts) return DPSNN_OK;
  const int rc = drain_bins(n, n->rate_first[k], nb, n->mbase[k], n->T[k].M, host_counts);
  if (rc != DPSNN_OK) return rc;
  n->rate_first[k] = done;
  return DPSNN_OK;
}

int dpsnn_stats(dpsnn_net* n, dpsnn_stats_t* out) {
  if (!n || !out) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  unsigned long long ns = 0;
  HIP_OK(hipMemcpy(&ns, n->sa.n_spikes, 8, hipMemcpyDeviceToHost));
  memset(out, 0, sizeof(*out));
  out->t = n->t;
  out->n_neurons = n->N_total;
  out->n_modules = n->M_total;
  out->n_synapses = n->N_total * n->p[0].K_out;
  out->n_spikes = (int64_t)ns;
  out->n_events = (int64_t)ns * n->p[0].K_out;
  out->build_ms = n->build_ms;
  out->bytes_rows = n->bytes_rows;
  out->bytes_state = n->bytes_state;
  out->bytes_total = n->bytes_total;
  {
    const int ab = acc_bytes(n->p[0]);
    out->lds_bytes = n->sched == DPSNN_SCHED_SPLIT
                         ? (int32_t)deliver_lds_bytes(n->sa, ab * 8)
                         : 1024 * 4 + 1024 * ab + kQueueMaxSlots * 4 + 4 * 256 * 4 + 16;
  }
  out->schedule = n->sched;
  out->n_index = n->N_index;
  out->n_nets = (int32_t)n->p.size();
  out->queue_cap = n->sa.q_cap;
  out->deliver_blocks = n->sa.deliver_blocks;
  out->route_blocks = n->sa.route_blocks;
  out->spike_lists = n->sa.spk_lists;
  out->n_pops = n->sa.P;
  out->queue_entry_bytes = n->sa.q_cap == 0 ? 0
                           : n->sa.q_code || n->sa.q_packed ? 4
                           : (acc_bytes(n->p[0]) == 4 ? (int32_t)sizeof(QEntry<int32_t>)
                                                      : (int32_t)sizeof(QEntry<int64_t>));
  return DPSNN_OK;
}

int dpsnn_stats_get(dpsnn_net* n, dpsnn_stats_t* out) { return dpsnn_stats(n, out); }

void dpsnn_free(dpsnn_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  drop_graph(n);
  release_all(n);
  delete n;
}

const char* dpsnn_strerror(int code) {
  switch (code) {
    case DPSNN_OK: return "ok";
    case DPSNN_E_INVAL: return "invalid argument";
    case DPSNN_E_NOMEM: return "out of memory";
    case DPSNN_E_DEVICE: return "HIP runtime error";
    case DPSNN_E_RANGE: return "fixed-point range exceeded";
    case DPSNN_E_SPIKELOG_FULL: return "spike log full";
    case DPSNN_E_STATE: return "invalid state";
    case DPSNN_E_RATES_FULL: return "rate bins full";
    case DPSNN_E_SCRATCH: return "request exceeds the fixed scratch buffer";
    default: return "unknown error";
  }
}

int dpsnn_read_state(dpsnn_net* n, float* V, float* c, uint8_t* ref) {
  if (!n) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  const size_t N = (size_t)n->N_index;
  if (V) HIP_OK(hipMemcpy(V, n->sa.V, N * 4, hipMemcpyDeviceToHost));
  if (c) HIP_OK(hipMemcpy(c, n->sa.c, N * 4, hipMemcpyDeviceToHost));
  if (ref) HIP_OK(hipMemcpy(ref, n->sa.ref, N, hipMemcpyDeviceToHost));
  return DPSNN_OK;
}

int dpsnn_write_state(dpsnn_net* n, const float* V, const float* c, const uint8_t* ref) {
  if (!n) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  const size_t N = (size_t)n->N_index;
  if (V) HIP_OK(hipMemcpy(n->sa.V, V, N * 4, hipMemcpyHostToDevice));
  if (c) HIP_OK(hipMemcpy(n->sa.c, c, N * 4, hipMemcpyHostToDevice));
  if (ref) HIP_OK(hipMemcpy(n->sa.ref, ref, N, hipMemcpyHostToDevice));
  return DPSNN_OK;
}

int dpsnn_read_slots(dpsnn_net* n, int64_t* host_slots) {
  if (!n || !host_slots) return DPSNN_E_INVAL;
  HIP_OK(launch_drain(n->sa, n->p[0].acc_bits, (uint32_t)n->t, n->stream));
  HIP_OK(hipStreamSynchronize(n->stream));
  const int64_t N = n->N_index, Np = n->N_pad;
  const int ab = acc_bytes(n->p[0]);
  std::vector<unsigned char> buf((size_t)n->T[0].D * Np * ab);
  HIP_OK(hipMemcpy(buf.data(), n->sa.slots, buf.size(), hipMemcpyDeviceToHost));
  for (int64_t s = 0; s < n->T[0].D; ++s)
    for (int64_t i = 0; i < N; ++i) {
      const size_t at = (size_t)(s * Np + i);
      if (ab == 4) {
        int32_t v;
        memcpy(&v, &buf[at * 4], 4);
        host_slots[s * N + i] = v;
      } else {
        int64_t v;
        memcpy(&v, &buf[at * 8], 8);
        host_slots[s * N + i] = v;
      }
    }
  return DPSNN_OK;
}

int dpsnn_read_log(dpsnn_net* n, int32_t* host_step, int32_t* host_id, int64_t cap,
                   int64_t* n_out) {
  if (!n || !n_out || cap < 0) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  unsigned long long cnt = 0;
  const int rc = log_count(n, &cnt);
  if (rc != DPSNN_OK) return rc;
  const int64_t have = std::min<int64_t>((int64_t)cnt, n->p[0].spike_log_cap);
  *n_out = have;
  if (cap < have || have == 0 || !host_step || !host_id) return DPSNN_OK;
  std::vector<int2> buf((size_t)have);
  HIP_OK(hipMemcpy(buf.data(), n->sa.log, (size_t)have * 8, hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < have; ++k) {
    host_step[k] = buf[(size_t)k].x;
    host_id[k] = buf[(size_t)k].y;
  }
  return DPSNN_OK;
}

int dpsnn_read_rows(dpsnn_net* n, int64_t first, int64_t count, int32_t* host_tgt, void* host_w,
                    uint8_t* host_dk) {
  if (!n || first < 0 || count < 0 || first + count > n->N_index) return DPSNN_E_INVAL;
  HIP_OK(hipStreamSynchronize(n->stream));
  const int Ko = n->p[0].K_out, rs = n->T[0].row_stride;
  const int wb = w_bytes(n->p[0]);
  if ((host_tgt || host_dk) && Ko > 0 && count > 0) {
    std::vector<int32_t> words((size_t)count * Ko);
    HIP_OK(hipMemcpy2D(words.data(), (size_t)Ko * 4, n->sa.tgt + first * rs, (size_t)rs * 4,
                       (size_t)Ko * 4, (size_t)count, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < words.size(); ++k) {
      if (host_tgt) host_tgt[k] = words[k] & kTargetMask;
      if (host_dk) host_dk[k] = (uint8_t)((uint32_t)words[k] >> kDelayShift);
    }
  }
  if (host_w && Ko > 0 && count > 0)
    HIP_OK(hipMemcpy2D(host_w, (size_t)Ko * wb,
                       static_cast<const unsigned char*>(n->sa.w) + (size_t)first * rs * wb,
                       (size_t)rs * wb, (size_t)Ko * wb, (size_t)count, hipMemcpyDeviceToHost));
  return DPSNN_OK;
}

int dpsnn_read_plasticity(dpsnn_net* n, int64_t first, int64_t count, int32_t* host_t_act,
                          float* host_y) {
  if (!n || first < 0 || count < 0 || first + count > n->N_index) return DPSNN_E_INVAL;
  if (!n->sa.plastic) return DPSNN_E_STATE;
  HIP_OK(hipStreamSynchronize(n->stream));
  const int Ko = n->p[0].K_out, rs = n->T[0].row_stride;
  if (Ko == 0 || count == 0) return DPSNN_OK;
  if (host_t_act)
    HIP_OK(hipMemcpy2D(host_t_act, (size_t)Ko * 4, n->sa.syn_t + first * rs, (size_t)rs * 4,
                       (size_t)Ko * 4, (size_t)count, hipMemcpyDeviceToHost));
  if (host_y)
    HIP_OK(hipMemcpy2D(host_y, (size_t)Ko * 4, n->sa.syn_y + first * rs, (size_t)rs * 4,
                       (size_t)Ko * 4, (size_t)count, hipMemcpyDeviceToHost));
  return DPSNN_OK;
}

int64_t dpsnn_host_table(const dpsnn_params* p, const char* name, void* out, int64_t cap) {
  if (!p || !name) return DPSNN_E_INVAL;
  HostTables T;
  const int rc = compute_tables(*p, T);
  if (rc != DPSNN_OK) return rc;
  if (!strncmp(name, "wfix_", 5)) {  // wfix_<q> (block 0) or wfix_<q>_<b>
    const char* d = name + 5;
    int q = -1, b = 0;
    if (strlen(d) == 1 && d[0] >= '0' && d[0] <= '3') {
      q = d[0] - '0';
    } else if (strlen(d) == 3 && d[0] >= '0' && d[0] <= '3' && d[1] == '_' && d[2] >= '0' &&
               d[2] <= '3') {
      q = d[0] - '0';
      b = d[2] - '0';
    }
    if (q < 0 || q >= T.P || b >= T.tables(q)) return DPSNN_E_INVAL;
    std::vector<int64_t> v = fix_table(*p, T, q, b);
    const int64_t bytes = (int64_t)v.size() * 8;
    if (out && cap >= bytes) memcpy(out, v.data(), (size_t)bytes);
    return bytes;
  }
  return host_table(T, name, out, cap);
}

int dpsnn_waves(dpsnn_net* n, const dpsnn_wave_params* wp, dpsnn_wave_result* out,
                int32_t* host_tr_module, double* host_tr_T, int32_t* host_tr_wave,
                int64_t cap_tr, double* host_wave_speed, double* host_wave_t0,
                int32_t* host_wave_n, int64_t cap_waves) {
  if (!n || !wp || !out || wp->net < 0 || wp->net >= (int32_t)n->p.size() || wp->n_bins < 0)
    return DPSNN_E_INVAL;
  const int64_t done = n->t / n->p[0].rate_bin_steps;
  const int64_t avail = done - n->rate_first[wp->net];
  if (avail < 1) return DPSNN_E_STATE;
  const int64_t nb = wp->n_bins > 0 ? std::min<int64_t>(wp->n_bins, avail) : avail;
  if (nb > kWaveMaxBins) return DPSNN_E_INVAL;
  const dpsnn_params& q = n->p[wp->net];
  WaveArgs a{};
  a.counts = n->sa.rates;
  a.ring = n->p[0].rate_bins_cap;
  a.M_stride = n->M_total;
  a.mbase = n->mbase[wp->net];
  a.bin0 = done - nb;
  a.slot0 = a.bin0 % a.ring;
  a.nb = (int32_t)nb;
  a.W = q.grid_w;
  a.H = q.grid_h;
  a.M = q.grid_w * q.grid_h;
  a.P = n->sa.P;
  Scratch S;
  S.free_fn = n->free_fn;
  S.ctx = n->alloc_ctx;
  return waves_impl(a, n->p[0].rate_bin_steps, n->p[0].dt_ms, wp, n->stream, S, nullptr, 0,
                    out,
                    host_tr_module, host_tr_T, host_tr_wave, cap_tr, host_wave_speed,
                    host_wave_t0, host_wave_n, cap_waves);
}

int dpsnn_waves_counts(const uint32_t* dev_counts, int64_t n_bins, int32_t grid_w,
                       int32_t grid_h, int32_t n_pops, int32_t bin_steps, double dt_ms,
                       int64_t bin0, const dpsnn_wave_params* wp, void* stream,
                       dpsnn_wave_result* out, int32_t* host_tr_module, double* host_tr_T,
                       int32_t* host_tr_wave, int64_t cap_tr, double* host_wave_speed,
                       double* host_wave_t0, int32_t* host_wave_n, int64_t cap_waves) {
  if (!dev_counts || n_bins < 1 || n_bins > kWaveMaxBins || grid_w < 1 || grid_h < 1 ||
      bin0 < 0 || (int64_t)grid_w * grid_h > kWaveMaxModules)
    return DPSNN_E_INVAL;
  WaveArgs a{};
  a.counts = dev_counts;
  a.ring = n_bins;
  a.M_stride = (int64_t)grid_w * grid_h;
  a.mbase = 0;
  a.slot0 = 0;  // the window is the whole buffer
  a.bin0 = bin0;
  a.nb = (int32_t)n_bins;
  a.W = grid_w;
  a.H = grid_h;
  a.M = grid_w * grid_h;
  a.P = n_pops;
  Scratch S;
  return waves_impl(a, bin_steps, dt_ms, wp, static_cast<hipStream_t>(stream), S, nullptr,
                    0, out,
                    host_tr_module, host_tr_T, host_tr_wave, cap_tr, host_wave_speed,
                    host_wave_t0, host_wave_n, cap_waves);
}


int dpsnn_waves_counts_static(const uint32_t* dev_counts, int64_t n_bins, int32_t grid_w,
                              int32_t grid_h, int32_t n_pops, int32_t bin_steps, double dt_ms,
                              int64_t bin0, const dpsnn_wave_params* wp, void* stream,
                              dpsnn_wave_result* out, int32_t* host_tr_module,
                              double* host_tr_T, int32_t* host_tr_wave, int64_t cap_tr,
                              double* host_wave_speed, double* host_wave_t0,
                              int32_t* host_wave_n, int64_t cap_waves) {
  if (!dev_counts || n_bins < 1 || n_bins > kWaveMaxBins || grid_w < 1 || grid_h < 1 ||
      bin0 < 0 || (int64_t)grid_w * grid_h > kWaveMaxModules)
    return DPSNN_E_INVAL;
  WaveArgs a{};
  a.counts = dev_counts;
  a.ring = n_bins;
  a.M_stride = (int64_t)grid_w * grid_h;
  a.mbase = 0;
  a.slot0 = 0;
  a.bin0 = bin0;
  a.nb = (int32_t)n_bins;
  a.W = grid_w;
  a.H = grid_h;
  a.M = grid_w * grid_h;
  a.P = n_pops;
  int rc = waves_check(a, bin_steps, dt_ms, wp, out, cap_tr, cap_waves);
  if (rc != DPSNN_OK) return rc;
  // the buffers this request needs, counted before any device call
  {
    WaveArgs m = a;
    WaveBufs B{};
    Scratch count;
    count.measure = true;
    rc = waves_take(m, wp, kWaveScratchMaxCount + 2, count, B);
    if (rc != DPSNN_OK) return rc;
    if (count.used > kWaveScratchBytes) return DPSNN_E_SCRATCH;
  }
  void* base = nullptr;
  const double* lnt = nullptr;
  rc = scratch_setup(&base, &lnt);
  if (rc != DPSNN_OK) return rc;
  Scratch S;
  S.arena = static_cast<unsigned char*>(base);
  S.arena_cap = kWaveScratchBytes;
  rc = waves_impl(a, bin_steps, dt_ms, wp, static_cast<hipStream_t>(stream), S, lnt,
                  kWaveScratchMaxCount + 2, out, host_tr_module, host_tr_T, host_tr_wave,
                  cap_tr, host_wave_speed, host_wave_t0, host_wave_n, cap_waves);
  return rc == DPSNN_E_NOMEM ? DPSNN_E_SCRATCH : rc;
}

}  // extern "C"
