// Batched path: many instances of uneven (N, P) in one launch sequence.
//
// The instances advance in lock step over a global pivot counter: every launch
// covers all instances that still have work at that step (argument records in
// a device table, one per instance), so the sequential chain of Algorithm 1 is
// paid once for the batch instead of once per instance.  The trailing update of
// all instances at a panel step is one persistent MFMA launch fed from 8 per-XCD
// queues of work items, largest first (Section 4.3.3 distributes the largest
// work first for the same reason).  The whole sequence -- load, panels, the
// first k columns of L^-1, the blocks and the eigen-steps -- is captured once in
// a hipGraph and replayed; dependencies between steps are graph edges (stream
// order), so no kernel ever waits on another workgroup.
//
// Tuning knobs (hl_tune_t) change only the launch shape, never the bits: the
// work-item granularity of the MFMA launches and the form (MFMA or VALU) of
// small-precision instances.  hl_autotune times candidate settings on the
// batch's first panel steps and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hl_host.hpp"
#include "hl_kernels.hpp"

using namespace hl;

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) return fail(HL_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

namespace {

// host image of the device plan buffer: records appended with 16-byte alignment
struct Blob {
  std::vector<char> bytes;
  template <class T>
  size_t put(const std::vector<T>& v) {
    size_t off = (bytes.size() + 15) / 16 * 16;
    bytes.resize(off + v.size() * sizeof(T));
    if (!v.empty()) memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  size_t reserve(size_t n) {
    size_t off = (bytes.size() + 15) / 16 * 16;
    bytes.resize(off + n);
    return off;
  }
};

struct Inst {
  hl_instance in;
  Dims dm;
  Layout L;
  int form;  // trailing-update form used in the batch
  int kara;  // Karatsuba levels of its trailing updates (MFMA form; 0: the digit product)
  char* base;
  DevStatus* st;
  u32 *A, *up, *omega;
  size_t ldb, ldx;
};

// One recorded launch; offsets point into the plan buffer.
struct Op {
  enum Kind {
    FILL, SCALES, LOAD, PIVOT, COL, VALU, RECODE, MFMA, CARRY, TRSM_ROW, BLOCK, EIG, COLU, COLFIN, TOEP, BLOCKY,
    BLOCKSUM, KARA_PREP, KARA_FIN
  } kind;
  int inst = -1;           // FILL, SCALES, LOAD, BLOCK: the instance
  size_t off = 0;          // table offset
  size_t off2 = 0;         // MFMA: items
  int count = 0;           // records
  int a = 0, b = 0, c = 0, d = 0;  // launch extents (see issue())
  u32* fp = nullptr;       // FILL target
  size_t fn = 0;           // FILL words
  size_t x[4] = {0, 0, 0, 0};  // TOEP: recode threads (b, u), work items, entries
  KaraArgs ka{};           // KARA_PREP, KARA_FIN: the instance's Karatsuba record
  RangeTab rt{};           // KARA_FIN: its ranges (a = C_lo, b = tiles)
};

// one batched Toeplitz-form launch set over prepared records
void put_toep(Blob& blob, std::vector<Op>& ops, const std::vector<ToepArgs>& v) {
  if (v.empty()) return;
  Op o;
  o.kind = Op::TOEP;
  for (const ToepArgs& a : v) {
    size_t e[4];
    toep_extents(a, &e[0], &e[1], &e[2], &e[3]);
    for (int q = 0; q < 4; ++q) o.x[q] = std::max(o.x[q], e[q]);
    o.a = std::max(o.a, a.nrg);
  }
  o.off = blob.put(v);
  o.count = (int)v.size();
  ops.push_back(o);
}

// prepare a record and keep it if it has work
hl_status add_toep(std::vector<ToepArgs>& v, ToepArgs a) {
  bool empty = false;
  const hipError_t e = toep_prepare(a, &empty);
  if (e != hipSuccess) return fail(HL_EHIP, "Toeplitz update record: %s", hipGetErrorString(e));
  if (!empty) v.push_back(a);
  return HL_OK;
}

// cost of one work item of range rg of an MFMA entry, in MFMA steps
double item_cost(const RangeTab& rt, int rg, int S) {
  double c = 0;
  for (int tb = rt.tb[rg]; tb < rt.tb[rg + 1]; ++tb) {
    const int t0 = MF_BLOCK_DIGITS * tb;
    int jlo = t0 - (S - 1);
    if (jlo < 0) jlo = 0;
    jlo &= ~1;
    int jhi = t0 + MF_BLOCK_DIGITS - 1;
    if (jhi > S - 1) jhi = S - 1;
    const int nsteps = (jhi - jlo) / 2 + 1;
    c += (double)((nsteps + 9) / 10 * 10) + 8.0;
  }
  return c;
}

}  // namespace

struct hl_batch {
  hl_ctx* ctx = nullptr;
  std::vector<Inst> inst;
  hl_tune_t tune{};
  char* plan = nullptr;
  size_t plan_bytes = 0;
  size_t plan_used = 0;
  std::vector<Op> ops;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int steps = 0;  // panel steps recorded (for partial plans of the autotuner)
  int nl_max = 0;
};

namespace {

hl_status make_inst(const hl_instance& in, Inst* o) {
  hl_status s = make_dims(&in.shape, &o->dm);
  if (s != HL_OK) return s;
  if (!in.mu || !in.mu_exp || in.w < 1 || !in.ws || !in.f.d || !in.f.h || !in.f.s || !in.f.l || !in.x ||
      !in.blk || !in.blk_exp)
    return fail(HL_EINVAL, "batch instance with a null pointer");
  o->in = in;
  o->L = make_layout(o->dm);
  if (in.ws_bytes < o->L.total) return fail(HL_ENOMEM, "batch instance workspace %zu < %zu", in.ws_bytes, o->L.total);
  o->base = (char*)in.ws;
  o->st = (DevStatus*)(o->base + o->L.status);
  o->A = (u32*)(o->base + o->L.tiles);
  o->up = (u32*)(o->base + o->L.upanel);
  o->omega = (u32*)(o->base + o->L.omega);
  o->ldb = (size_t)o->dm.NT * o->dm.nl;
  o->ldx = (size_t)o->dm.k * o->dm.nl;
  return HL_OK;
}

MfmaArgs mfma_args(const Inst& I, const UpdArgs& g, int u_rows) {
  MfmaArgs m{};
  m.g = g;
  m.bdig = (int8_t*)(I.base + I.L.bdig);
  m.udig = (int8_t*)(I.base + I.L.udig);
  m.slices = I.L.digit_slices;
  m.pad = kDigitPad;
  m.S = I.dm.S;
  m.NT = I.dm.NT;
  m.carry = (long long*)(I.base + I.L.carry);
  m.max_ranges = kMaxRanges;
  m.carry_tiles = I.L.carry_tiles;
  m.timing = nullptr;
  m.u_rows = u_rows;
  return m;
}

// Karatsuba record of an instance's update g (as hl_factor builds it)
KaraArgs kara_args(const Inst& I, const UpdArgs& g, int u_rows) {
  KaraArgs ka{};
  ka.m = mfma_args(I, g, u_rows);
  ka.m.S = I.dm.Sk0;
  ka.levels = I.kara;
  for (int lv = 1; lv <= I.kara; ++lv) {
    ka.pan[lv] = (int8_t*)(I.base + I.L.kara_pan[lv]);
    ka.pan_stride[lv] = I.L.kara_pan_bytes[lv];
    ka.pan_slices[lv] = I.L.kara_pan_slices[lv];
  }
  ka.Sk = kara_leaf_digits(I.dm.Sk0, I.kara);
  ka.kslices = ka.Sk + 2 * kDigitPad;
  ka.prod = (u32*)(I.base + I.L.kara_prod);
  ka.nwp = kara_nwp(I.dm.Sk0, I.kara);
  ka.prod_tiles = I.L.kara_tiles;
  return ka;
}

// Work items of one step's MFMA entries into 8 per-XCD queues.  Bundles are the
// tiles of one (entry, range), cut into chunks of at most 128 items (one round of
// an XCD); chunks go to the least loaded XCD, largest item cost first.
void build_queues(const std::vector<MfmaEntry>& ents, int items_per_simd, std::vector<MfmaEntry>* out_ents,
                  std::vector<int4>* items, int* per_xcd) {
  (void)items_per_simd;
  struct Chunk {
    int e, rg, lt0, lt1;
    double cost;  // per item
  };
  std::vector<Chunk> chunks;
  for (int e = 0; e < (int)ents.size(); ++e) {
    const MfmaEntry& E = ents[e];
    for (int rg = 0; rg < E.rt.n; ++rg) {
      const double c = item_cost(E.rt, rg, E.m.S);
      for (int lt = 0; lt < E.ntiles; lt += 128) chunks.push_back({e, rg, lt, std::min(E.ntiles, lt + 128), c});
    }
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& a, const Chunk& b) { return a.cost > b.cost; });
  double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<std::vector<int4>> q(8);
  for (const Chunk& c : chunks) {
    int x = 0;
    for (int j = 1; j < 8; ++j)
      if (load[j] < load[x]) x = j;
    for (int lt = c.lt0; lt < c.lt1; ++lt) q[x].push_back(make_int4(c.e, lt, c.rg, 0));
    load[x] += c.cost * (c.lt1 - c.lt0);
  }
  int per = 0;
  for (auto& v : q) per = std::max(per, (int)v.size());
  items->assign((size_t)8 * per, make_int4(-1, 0, 0, 0));
  for (int x = 0; x < 8; ++x)
    for (size_t k = 0; k < q[x].size(); ++k) (*items)[(size_t)x * per + k] = q[x][k];
  *per_xcd = per;
  *out_ents = ents;
}

// number of ranges of an entry: items of about 1 / (items_per_simd * 1024) of
// the step's MFMA work, within the range cap and the carry capacity
int pick_ranges(double tile_cost, double step_cost, int ntiles, int ntb, const hl_tune_t& t, size_t carry_tiles) {
  const double target = step_cost / (1024.0 * std::max(1, t.items_per_simd));
  int n = (int)std::ceil(tile_cost / std::max(1.0, target));
  n = std::max(1, std::min(n, std::min(t.range_cap > 0 ? t.range_cap : kMaxRanges, std::min(MF_MAX_RANGES, ntb))));
  while (n > 1 && (size_t)ntiles * n > carry_tiles) --n;
  return n;
}

// Record one trailing (or triangular-solve) update step for the instances in
// `who`, with UpdArgs g_of(i) and panel digit sources; appends ops.
struct StepUpd {
  int i;
  UpdArgs g;
  const u32* bsrc;
  size_t blds;
  const u32* usrc;
  size_t ulds;
  int u_rows;
  int C_lo, nrow, ncol, ntiles;
};

void record_update_step(hl_batch* B, Blob& blob, std::vector<StepUpd>& ups) {
  // VALU-form instances
  std::vector<UpdArgs> vt;
  int nr = 0, nc = 0, nwm = 0, nlm = 0;
  // MFMA-form instances: digit-product entries first (their carries are added
  // into the targets by k_carry_fix_b), then the Karatsuba products
  std::vector<RecodeArgs> rc;
  std::vector<MfmaEntry> ents, kents;
  std::vector<Op> kprep, kfin;
  int NTm = 0, nrowm = 0, ncolm = 0;
  double step_cost = 0;
  // per update: the cost of one work item covering a whole tile (of one product
  // for the Karatsuba form), its records
  std::vector<double> tile_cost(ups.size(), 0.0);
  std::vector<KaraArgs> kas(ups.size());
  for (size_t j = 0; j < ups.size(); ++j) {
    const Inst& I = B->inst[ups[j].i];
    if (I.form != HL_FORM_MFMA8) continue;
    if (I.kara > 0) {
      kas[j] = kara_args(I, ups[j].g, ups[j].u_rows);
      const RangeTab one = split_ranges_ntb(kas[j].nwp / 4, kas[j].Sk, 1);
      tile_cost[j] = item_cost(one, 0, kas[j].Sk);
      step_cost += tile_cost[j] * ups[j].ntiles * kara_products(I.kara);
    } else {
      const RangeTab one = split_ranges(I.dm.nl, I.dm.S, 1);
      tile_cost[j] = item_cost(one, 0, I.dm.S);
      step_cost += tile_cost[j] * ups[j].ntiles;
    }
  }
  for (size_t j = 0; j < ups.size(); ++j) {
    const StepUpd& u = ups[j];
    const Inst& I = B->inst[u.i];
    if (I.form != HL_FORM_MFMA8) {
      vt.push_back(u.g);
      nr = std::max(nr, u.g.r_hi - u.g.r_lo);
      nc = std::max(nc, u.g.c_hi - u.g.c_lo);
      nwm = std::max(nwm, I.dm.nw);
      nlm = std::max(nlm, I.dm.nl);
      continue;
    }
    if (I.kara > 0) {
      const KaraArgs& ka = kas[j];
      const int np = kara_products(I.kara);
      const int n = pick_ranges(tile_cost[j], step_cost, np * u.ntiles, ka.nwp / 4, B->tune, I.L.carry_tiles);
      const RangeTab rt = split_ranges_ntb(ka.nwp / 4, ka.Sk, n);
      for (int p = 0; p < np; ++p) {
        MfmaEntry E{};
        E.m = ka.m;
        E.m.bdig = ka.pan[I.kara] + (size_t)p * ka.pan_stride[I.kara];
        E.m.udig = ka.pan[I.kara] + (size_t)(np + p) * ka.pan_stride[I.kara];
        E.m.slices = ka.kslices;
        E.m.S = kara_prod_digits(ka.m.S, I.kara, p);  // its own operand length (<= Sk)
        E.m.carry = ka.m.carry + (size_t)p * u.ntiles * rt.n * 1024;
        E.rt = rt;
        E.C_lo = u.C_lo;
        E.ntiles = u.ntiles;
        E.store = ka.prod + (size_t)p * tile_words(ka.nwp);  // tile lt's products at lt np
        E.store_nw = ka.nwp;
        E.store_ts = (size_t)np * tile_words(ka.nwp);
        kents.push_back(E);
      }
      Op o;
      o.kind = Op::KARA_PREP;
      o.inst = u.i;
      o.ka = ka;
      kprep.push_back(o);
      o.kind = Op::KARA_FIN;
      o.rt = rt;
      o.a = u.C_lo;
      o.b = u.ntiles;
      kfin.push_back(o);
      continue;
    }
    rc.push_back(RecodeArgs{u.bsrc, u.blds, u.g.npan, I.dm.NT, I.dm.NT, I.dm.nl, kDigitPad,
                            (int8_t*)(I.base + I.L.bdig)});
    rc.push_back(RecodeArgs{u.usrc, u.ulds, u.g.npan, I.dm.NT, u.u_rows, I.dm.nl, kDigitPad,
                            (int8_t*)(I.base + I.L.udig)});
    NTm = std::max(NTm, I.dm.NT * I.dm.nl);  // recode threads / 16
    MfmaEntry E{};
    E.m = mfma_args(I, u.g, u.u_rows);
    const int n = pick_ranges(tile_cost[j], step_cost, u.ntiles, 8 * I.dm.nl / MF_BLOCK_DIGITS, B->tune,
                              I.L.carry_tiles);
    E.rt = split_ranges(I.dm.nl, I.dm.S, n);
    E.C_lo = u.C_lo;
    E.ntiles = u.ntiles;
    ents.push_back(E);
    nrowm = std::max(nrowm, u.nrow);
    ncolm = std::max(ncolm, u.ncol);
  }
  if (!vt.empty()) {
    Op o;
    o.kind = Op::VALU;
    o.off = blob.put(vt);
    o.count = (int)vt.size();
    o.a = nr;
    o.b = nc;
    o.c = nwm;
    o.d = nlm;
    B->ops.push_back(o);
  }
  if (!rc.empty()) {
    Op r;
    r.kind = Op::RECODE;
    r.off = blob.put(rc);
    r.count = (int)rc.size();
    r.a = NTm;
    B->ops.push_back(r);
  }
  for (const Op& o : kprep) B->ops.push_back(o);
  const int nd = (int)ents.size();
  ents.insert(ents.end(), kents.begin(), kents.end());
  if (!ents.empty()) {
    std::vector<MfmaEntry> e2;
    std::vector<int4> items;
    int per = 0;
    build_queues(ents, B->tune.items_per_simd, &e2, &items, &per);
    Op m;
    m.kind = Op::MFMA;
    m.off = blob.put(e2);
    m.off2 = blob.put(items);
    m.count = (int)e2.size();
    m.a = per;
    B->ops.push_back(m);
    if (nd > 0) {
      Op c;
      c.kind = Op::CARRY;
      c.off = m.off;  // the digit-product entries lead the table
      c.count = nd;
      c.a = nrowm;
      c.b = ncolm;
      B->ops.push_back(c);
    }
  }
  for (const Op& o : kfin) B->ops.push_back(o);
}

// Record the whole plan (max_panels < 0: everything; else only that many panel
// steps of the factorisation, for the autotuner).
hl_status record_plan(hl_batch* B, Blob& blob, int max_panels) {
  const int n = (int)B->inst.size();
  B->ops.clear();
  // --- load (per instance)
  for (int i = 0; i < n; ++i) {
    Inst& I = B->inst[i];
    Op f;
    f.kind = Op::FILL;
    f.fp = (u32*)I.st;
    f.fn = 64;
    B->ops.push_back(f);
    f.fp = I.in.f.l;
    f.fn = (size_t)I.dm.N * I.dm.NT * I.dm.nl;
    B->ops.push_back(f);
    f.fp = (u32*)(I.base + I.L.bdig);
    f.fn = (size_t)I.L.digit_slices * I.dm.NT * 4;
    B->ops.push_back(f);
    f.fp = (u32*)(I.base + I.L.udig);
    B->ops.push_back(f);
    for (int lv = 1; lv <= I.kara; ++lv) {
      // zero digit slices: the padding and the digits above the factors' read as zero
      f.fp = (u32*)(I.base + I.L.kara_pan[lv]);
      f.fn = 2 * kara_products(lv) * I.L.kara_pan_bytes[lv] / 4;
      B->ops.push_back(f);
    }
    Op s;
    s.kind = Op::SCALES;
    s.inst = i;
    B->ops.push_back(s);
    s.kind = Op::LOAD;
    B->ops.push_back(s);
  }
  // --- panels of Algorithm 1, all instances in lock step
  int Nmax = 0;
  for (auto& I : B->inst) Nmax = std::max(Nmax, I.dm.N);
  int panels = 0;
  for (int i0 = 0; i0 < Nmax; i0 += 16) {
    if (max_panels >= 0 && panels >= max_panels) break;
    ++panels;
    for (int il = 0; il < 16; ++il) {
      const int c = i0 + il;
      std::vector<PivotArgs> pv;
      std::vector<ColArgs> cl, cu;      // VALU-form column step; MFMA form: u_r
      std::vector<ColFinArgs> cf;       // MFMA form: rounding of the products
      std::vector<ToepArgs> tprod, tin; // MFMA form: column products, in-panel updates
      std::vector<UpdArgs> ip;
      int nlm = 0, rows = 0, nr = 0, nc = 0, nwm = 0, ldpm = 0;
      hl_status hs;
      for (int i = 0; i < n; ++i) {
        Inst& I = B->inst[i];
        if (c >= I.dm.N) continue;
        const int npan = std::min(16, I.dm.N - i0);
        pv.push_back(PivotArgs{I.A, I.dm, c, I.in.f.d, I.in.f.h, I.omega, I.L.omega_stride, I.st});
        const ColArgs ca{I.A, I.dm, c, i0, I.in.f.h, I.omega, I.L.omega_stride, I.up + (size_t)il * I.ldb,
                         I.in.f.l + (size_t)c * I.ldb, I.st};
        nlm = std::max(nlm, I.dm.nl);
        rows = std::max(rows, I.dm.NT - i0);
        if (I.form == HL_FORM_MFMA8) {
          // column step as in hl_factor: u_r, then P_r = u_r w_c as a Toeplitz
          // GEMM, then b_r = rnd(P_r / 2^P)
          u32* Pp = (u32*)(I.base + I.L.colprod);
          cu.push_back(ca);
          cf.push_back(ColFinArgs{ca, Pp, I.L.colprod_ld});
          ldpm = std::max(ldpm, I.L.colprod_ld);
          UpdArgs gp{};
          gp.A = Pp;
          gp.nw = I.L.colprod_ld;
          gp.nl = I.dm.nl;
          gp.Bop = ca.u_out;
          gp.Uop = I.omega + (size_t)c * I.L.omega_stride;
          gp.npan = 1;
          gp.r_lo = c + 1;
          gp.r_hi = I.dm.N;
          gp.c_lo = 0;
          gp.c_hi = 1;
          gp.st = I.st;
          ToepArgs tp = toep_args(gp, I.L, I.base, I.dm);
          tp.nlb = I.dm.nl;
          tp.nlu = I.dm.nl + 1;
          tp.plain = 1;
          tp.ldr = (size_t)I.L.colprod_ld;
          tp.add = 2;
          if ((hs = add_toep(tprod, tp)) != HL_OK) return hs;
        } else {
          cl.push_back(ca);
        }
        if (il + 1 < npan) {
          UpdArgs g{};
          g.A = I.A;
          g.tri = 1;
          g.nw = I.dm.nw;
          g.nl = I.dm.nl;
          g.Bop = I.in.f.l + (size_t)c * I.ldb;
          g.ldb = I.ldb;
          g.Uop = I.up + (size_t)il * I.ldb;
          g.ldu = I.ldb;
          g.npan = 1;
          g.r_lo = c + 1;
          g.r_hi = I.dm.N;
          g.c_lo = c + 1;
          g.c_hi = i0 + npan;
          g.st = I.st;
          if (I.form == HL_FORM_MFMA8) {
            if ((hs = add_toep(tin, toep_args(g, I.L, I.base, I.dm))) != HL_OK) return hs;
            continue;
          }
          ip.push_back(g);
          nr = std::max(nr, g.r_hi - g.r_lo);
          nc = std::max(nc, g.c_hi - g.c_lo);
          nwm = std::max(nwm, I.dm.nw);
        }
      }
      if (pv.empty()) break;
      Op o;
      o.kind = Op::PIVOT;
      o.off = blob.put(pv);
      o.count = (int)pv.size();
      o.d = nlm;
      B->ops.push_back(o);
      if (!cl.empty()) {
        o.kind = Op::COL;
        o.off = blob.put(cl);
        o.count = (int)cl.size();
        o.a = rows;
        B->ops.push_back(o);
      }
      if (!cu.empty()) {
        o.kind = Op::COLU;
        o.off = blob.put(cu);
        o.count = (int)cu.size();
        o.a = rows;
        B->ops.push_back(o);
        put_toep(blob, B->ops, tprod);
        Op f2;
        f2.kind = Op::COLFIN;
        f2.off = blob.put(cf);
        f2.count = (int)cf.size();
        f2.a = rows;
        f2.b = ldpm;
        B->ops.push_back(f2);
      }
      put_toep(blob, B->ops, tin);
      if (!ip.empty()) {
        Op v;
        v.kind = Op::VALU;
        v.off = blob.put(ip);
        v.count = (int)ip.size();
        v.a = nr;
        v.b = nc;
        v.c = nwm;
        v.d = nlm;
        B->ops.push_back(v);
      }
    }
    // trailing update of the panel
    std::vector<StepUpd> ups;
    for (int i = 0; i < n; ++i) {
      Inst& I = B->inst[i];
      if (i0 >= I.dm.N) continue;
      const int npan = std::min(16, I.dm.N - i0);
      if (i0 + npan >= I.dm.N) continue;
      StepUpd u{};
      u.i = i;
      u.g.A = I.A;
      u.g.tri = 1;
      u.g.nw = I.dm.nw;
      u.g.nl = I.dm.nl;
      u.g.Bop = I.in.f.l + (size_t)i0 * I.ldb;
      u.g.ldb = I.ldb;
      u.g.Uop = I.up;
      u.g.ldu = I.ldb;
      u.g.npan = npan;
      u.g.r_lo = i0 + npan;
      u.g.r_hi = I.dm.N;
      u.g.c_lo = i0 + npan;
      u.g.c_hi = I.dm.N;
      u.g.st = I.st;
      u.bsrc = u.g.Bop;
      u.blds = I.ldb;
      u.usrc = I.up;
      u.ulds = I.ldb;
      u.u_rows = I.dm.NT;
      u.C_lo = u.g.c_lo / 32;
      u.nrow = u.ncol = I.dm.nt - u.C_lo;
      u.ntiles = u.nrow * (u.nrow + 1) / 2;
      ups.push_back(u);
    }
    if (!ups.empty()) record_update_step(B, blob, ups);
  }
  B->steps = panels;
  if (max_panels >= 0) return HL_OK;

  // --- first k columns of L^-1 (Algorithm 4), all instances in lock step
  for (int i = 0; i < n; ++i) {
    Inst& I = B->inst[i];
    Op f;
    f.kind = Op::FILL;
    f.fp = I.A;
    f.fn = (size_t)I.dm.nt * tile_words(I.dm.nw);
    B->ops.push_back(f);
    f.fp = I.in.x;
    f.fn = (size_t)I.dm.NT * I.dm.k * I.dm.nl;
    B->ops.push_back(f);
    f.fp = (u32*)(I.base + I.L.bdig);
    f.fn = (size_t)I.L.digit_slices * I.dm.NT * 4;
    B->ops.push_back(f);
    f.fp = (u32*)(I.base + I.L.udig);
    B->ops.push_back(f);
  }
  for (int R0 = 0; R0 < Nmax; R0 += 16) {
    for (int j = 0; j < 16; ++j) {
      const int r = R0 + j;
      std::vector<TrsmRowArgs> tr;
      std::vector<UpdArgs> ib;
      std::vector<ToepArgs> tib;
      int km = 0, nlm = 0, nr = 0, nc = 0, nwm = 0;
      hl_status hs;
      for (int i = 0; i < n; ++i) {
        Inst& I = B->inst[i];
        if (r >= I.dm.N) continue;
        const int nb = std::min(16, I.dm.N - R0);
        tr.push_back(TrsmRowArgs{I.A, I.dm, r, I.in.f.s, I.in.f.h, I.in.x, I.st});
        km = std::max(km, I.dm.k);
        nlm = std::max(nlm, I.dm.nl);
        if (j + 1 < nb) {
          UpdArgs g{};
          g.A = I.A;
          g.tri = 0;
          g.ntc = 1;
          g.nw = I.dm.nw;
          g.nl = I.dm.nl;
          g.Bop = I.in.f.l + (size_t)r * I.ldb;
          g.ldb = I.ldb;
          g.Uop = I.in.x + (size_t)r * I.ldx;
          g.ldu = I.ldx;
          g.npan = 1;
          g.r_lo = r + 1;
          g.r_hi = R0 + nb;
          g.c_lo = 0;
          g.c_hi = I.dm.k;
          g.st = I.st;
          if (I.form == HL_FORM_MFMA8) {
            if ((hs = add_toep(tib, toep_args(g, I.L, I.base, I.dm))) != HL_OK) return hs;
            continue;
          }
          ib.push_back(g);
          nr = std::max(nr, g.r_hi - g.r_lo);
          nc = std::max(nc, g.c_hi - g.c_lo);
          nwm = std::max(nwm, I.dm.nw);
        }
      }
      if (tr.empty()) break;
      Op o;
      o.kind = Op::TRSM_ROW;
      o.off = blob.put(tr);
      o.count = (int)tr.size();
      o.a = km;
      o.d = nlm;
      B->ops.push_back(o);
      put_toep(blob, B->ops, tib);
      if (!ib.empty()) {
        Op v;
        v.kind = Op::VALU;
        v.off = blob.put(ib);
        v.count = (int)ib.size();
        v.a = nr;
        v.b = nc;
        v.c = nwm;
        v.d = nlm;
        B->ops.push_back(v);
      }
    }
    std::vector<ToepArgs> ttr;
    hl_status hs2;
    std::vector<StepUpd> ups;
    for (int i = 0; i < n; ++i) {
      Inst& I = B->inst[i];
      if (R0 >= I.dm.N) continue;
      const int nb = std::min(16, I.dm.N - R0);
      if (R0 + nb >= I.dm.N) continue;
      StepUpd u{};
      u.i = i;
      u.g.A = I.A;
      u.g.tri = 0;
      u.g.ntc = 1;
      u.g.nw = I.dm.nw;
      u.g.nl = I.dm.nl;
      u.g.Bop = I.in.f.l + (size_t)R0 * I.ldb;
      u.g.ldb = I.ldb;
      u.g.Uop = I.in.x + (size_t)R0 * I.ldx;
      u.g.ldu = I.ldx;
      u.g.npan = nb;
      u.g.r_lo = R0 + nb;
      u.g.r_hi = I.dm.N;
      u.g.c_lo = 0;
      u.g.c_hi = I.dm.k;
      u.g.st = I.st;
      u.bsrc = u.g.Bop;
      u.blds = I.ldb;
      u.usrc = u.g.Uop;
      u.ulds = I.ldx;
      u.u_rows = I.dm.k;
      u.C_lo = u.g.r_lo / 32;
      u.nrow = I.dm.nt - u.C_lo;
      u.ncol = 1;
      u.ntiles = u.nrow;
      if (I.form == HL_FORM_MFMA8) {
        // k <= 32 target columns: the Toeplitz form keeps every MFMA column busy
        if ((hs2 = add_toep(ttr, toep_args(u.g, I.L, I.base, I.dm))) != HL_OK) return hs2;
        continue;
      }
      ups.push_back(u);
    }
    put_toep(blob, B->ops, ttr);
    if (!ups.empty()) record_update_step(B, blob, ups);
  }
  // --- blocks and eigen-steps (one launch).  MFMA form as in hl_inv_block:
  // y = x w per instance, the sums over r as Toeplitz GEMMs of rank 16 in lock
  // step over all instances, then gather, reduction and rounding per instance
  std::vector<EigArgs> eg;
  int nlm = 0;
  for (int i = 0; i < n; ++i) {
    Op b;
    b.kind = B->inst[i].form == HL_FORM_MFMA8 ? Op::BLOCKY : Op::BLOCK;
    b.inst = i;
    B->ops.push_back(b);
    Inst& I = B->inst[i];
    eg.push_back(eig_args(I.in.blk, I.dm, I.base + I.L.eig, I.st));
    nlm = std::max(nlm, I.dm.nl);
  }
  for (int r0 = 0; r0 < Nmax; r0 += 16) {
    std::vector<ToepArgs> tb;
    for (int i = 0; i < n; ++i) {
      Inst& I = B->inst[i];
      if (I.form != HL_FORM_MFMA8 || r0 >= I.dm.N) continue;
      UpdArgs g{};
      g.A = (u32*)(I.base + I.L.blk_m);
      g.tri = 1;
      g.nw = I.L.blk_nm;
      g.nl = I.dm.nl;
      g.Bop = (u32*)(I.base + I.L.blk_y) + (size_t)r0 * I.L.blk_ny;
      g.ldb = I.L.blk_ny;
      g.rsb = (size_t)I.dm.NT * I.L.blk_ny;
      g.Uop = I.in.x + (size_t)r0 * I.ldx;
      g.ldu = I.ldx;
      g.npan = std::min(16, I.dm.N - r0);
      g.r_lo = 0;
      g.r_hi = I.dm.k;
      g.c_lo = 0;
      g.c_hi = I.dm.k;
      g.st = I.st;
      ToepArgs ta = toep_args(g, I.L, I.base, I.dm);
      ta.NT = 32;
      ta.nlb = 2 * I.dm.nl + 1;
      ta.nlu = I.dm.nl;
      ta.ucs = (size_t)I.dm.nl;
      ta.plain = 1;
      ta.ldr = (size_t)I.dm.k * I.L.blk_nm;
      ta.ldc = (size_t)I.L.blk_nm;
      ta.add = 1;
      hl_status hs3 = add_toep(tb, ta);
      if (hs3 != HL_OK) return hs3;
    }
    put_toep(blob, B->ops, tb);
  }
  for (int i = 0; i < n; ++i) {
    if (B->inst[i].form != HL_FORM_MFMA8) continue;
    Op b;
    b.kind = Op::BLOCKSUM;
    b.inst = i;
    B->ops.push_back(b);
  }
  Op e;
  e.kind = Op::EIG;
  e.off = blob.put(eg);
  e.count = n;
  e.d = nlm;
  B->ops.push_back(e);
  return HL_OK;
}

hl_status issue(hl_batch* B, hipStream_t st) {
  char* P = B->plan;
  // the 8 queue heads of the MFMA launches sit at the start of the plan buffer
  unsigned* heads = (unsigned*)P;
  for (const Op& o : B->ops) {
    switch (o.kind) {
      case Op::FILL:
        HIPCHK(launch_fill(o.fp, o.fn, 0u, st));
        break;
      case Op::SCALES: {
        const Inst& I = B->inst[o.inst];
        HIPCHK(launch_scales(I.in.mu, I.in.mu_exp, I.in.w, I.dm.N, I.dm.E, I.in.f.s, I.st, st));
        break;
      }
      case Op::LOAD: {
        const Inst& I = B->inst[o.inst];
        HIPCHK(launch_load(I.in.mu, I.in.mu_exp, I.in.w, I.in.f.s, I.dm, I.A, I.st, st));
        break;
      }
      case Op::PIVOT:
        HIPCHK(launch_pivot_batch((const PivotArgs*)(P + o.off), o.count, o.d, st));
        break;
      case Op::COL:
        HIPCHK(launch_col_batch((const ColArgs*)(P + o.off), o.count, o.a, o.d, st));
        break;
      case Op::VALU:
        HIPCHK(launch_upd_valu_batch((const UpdArgs*)(P + o.off), o.count, o.a, o.b, o.c, o.d, st));
        break;
      case Op::RECODE:
        HIPCHK(launch_recode_batch((const RecodeArgs*)(P + o.off), o.count, o.a, st));
        break;
      case Op::MFMA:
        HIPCHK(launch_upd_mfma_batch((const MfmaEntry*)(P + o.off), (const int4*)(P + o.off2), o.a, heads, st));
        break;
      case Op::CARRY:
        HIPCHK(launch_carry_fix_batch((const MfmaEntry*)(P + o.off), o.count, o.a, o.b, st));
        break;
      case Op::TRSM_ROW:
        HIPCHK(launch_trsm_row_batch((const TrsmRowArgs*)(P + o.off), o.count, o.a, o.d, st));
        break;
      case Op::BLOCK: {
        const Inst& I = B->inst[o.inst];
        HIPCHK(launch_block(I.in.x, I.dm, I.omega, I.L.omega_stride, I.in.f.s, (u32*)(I.base + I.L.blk_part),
                            I.L.blk_stride, I.L.blk_chunks, kBlockRows, (u32*)(I.base + I.L.blk_sum),
                            I.L.blk_stride + 64, I.in.blk, I.in.blk_exp, I.st, st));
        break;
      }
      case Op::EIG:
        HIPCHK(launch_eig_batch((const EigArgs*)(P + o.off), o.count, o.d, st));
        break;
      case Op::BLOCKY: {
        const Inst& I = B->inst[o.inst];
        HIPCHK(launch_fill((u32*)(I.base + I.L.blk_m), (size_t)I.dm.k * I.dm.k * I.L.blk_nm, 0u, st));
        HIPCHK(launch_block_y(I.in.x, I.dm, I.omega, I.L.omega_stride, (u32*)(I.base + I.L.blk_y), I.L.blk_ny, I.st,
                              st));
        break;
      }
      case Op::BLOCKSUM: {
        const Inst& I = B->inst[o.inst];
        u32* part = (u32*)(I.base + I.L.blk_part);
        HIPCHK(launch_block_gather((const u32*)(I.base + I.L.blk_m), nullptr, I.L.blk_nm, I.dm, part, I.L.blk_stride, I.st,
                                   st));
        HIPCHK(launch_block_sums(I.dm, I.in.f.s, part, I.L.blk_stride, 1, (u32*)(I.base + I.L.blk_sum),
                                 I.L.blk_stride + 64, I.in.blk, I.in.blk_exp, I.st, st));
        break;
      }
      case Op::COLU:
        HIPCHK(launch_col_u_batch((const ColArgs*)(P + o.off), o.count, o.a, B->nl_max, st));
        break;
      case Op::COLFIN:
        HIPCHK(launch_col_fin_batch((const ColFinArgs*)(P + o.off), o.count, o.a, o.b, st));
        break;
      case Op::TOEP:
        HIPCHK(launch_upd_toep_batch((const ToepArgs*)(P + o.off), o.count, o.x[0], o.x[1], o.x[2], o.x[3], o.a, st));
        break;
      case Op::KARA_PREP:
        HIPCHK(launch_kara_prep(o.ka, st));
        break;
      case Op::KARA_FIN:
        HIPCHK(launch_kara_finish(o.ka, o.rt, o.a, o.b, st));
        break;
    }
  }
  return HL_OK;
}

hl_status build(hl_batch* B, int max_panels) {
  Blob blob;
  blob.reserve(256);  // queue heads
  hl_status s = record_plan(B, blob, max_panels);
  if (s != HL_OK) return s;
  if (blob.bytes.size() > B->plan_bytes)
    return fail(HL_ENOMEM, "batch plan needs %zu bytes, buffer has %zu", blob.bytes.size(), B->plan_bytes);
  B->plan_used = blob.bytes.size();
  HIPCHK(hipMemcpy(B->plan, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice));
  return HL_OK;
}

hl_status capture(hl_batch* B) {
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(HL_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  hl_status s = issue(B, cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (s != HL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(HL_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  B->graph = g;
  HIPCHK(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  return HL_OK;
}

hl_status init_batch(hl_ctx* ctx, int32_t count, const hl_instance* inst, const hl_tune_t* tune, void* plan,
                     size_t plan_bytes, hl_batch* B) {
  if (!ctx || count < 1 || !inst || !plan) return fail(HL_EINVAL, "bad batch arguments");
  B->ctx = ctx;
  B->plan = (char*)plan;
  B->plan_bytes = plan_bytes;
  B->tune = tune ? *tune : hl_tune_t{8, kMaxRanges, 0, 0};
  if (B->tune.items_per_simd < 1) B->tune.items_per_simd = 1;
  B->inst.resize(count);
  for (int i = 0; i < count; ++i) {
    hl_status s = make_inst(inst[i], &B->inst[i]);
    if (s != HL_OK) return fail(s, "instance %d: %s", i, hl_last_error());
    Inst& I = B->inst[i];
    I.form = I.in.shape.form;
    if (I.dm.P < B->tune.valu_below_bits) I.form = HL_FORM_VALU;
    I.kara = 0;
    if (I.form == HL_FORM_MFMA8) {
      const int want = B->tune.karatsuba == 0 ? kara_auto_level(I.dm.P) : std::max(0, B->tune.karatsuba);
      I.kara = std::min(want, I.dm.kara);
    }
    B->nl_max = std::max(B->nl_max, I.dm.nl);
  }
  return HL_OK;
}

}  // namespace

extern "C" hl_status hl_batch_plan_bytes(int32_t count, const hl_instance* inst, const hl_tune_t* tune,
                                         size_t* bytes) {
  if (!bytes) return fail(HL_EINVAL, "null output");
  hl_batch B;
  hl_ctx* dummy = (hl_ctx*)1;  // planning only: no device calls
  hl_status s = init_batch(dummy, count, inst, tune, (void*)1, 0, &B);
  if (s != HL_OK) return s;
  Blob blob;
  blob.reserve(256);
  s = record_plan(&B, blob, -1);
  if (s != HL_OK) return s;
  *bytes = blob.bytes.size();
  return HL_OK;
}

extern "C" hl_status hl_batch_create(hl_ctx* ctx, int32_t count, const hl_instance* inst, const hl_tune_t* tune,
                                     void* plan, size_t plan_bytes, hl_batch** out) {
  if (!out) return fail(HL_EINVAL, "null output");
  *out = nullptr;
  hl_batch* B = new hl_batch();
  hl_status s = init_batch(ctx, count, inst, tune, plan, plan_bytes, B);
  if (s == HL_OK) s = build(B, -1);
  if (s == HL_OK) s = capture(B);
  if (s != HL_OK) {
    hl_batch_destroy(B);
    return s;
  }
  *out = B;
  return HL_OK;
}

extern "C" hl_status hl_batch_launch(hl_batch* B, void* stream) {
  if (!B || !B->exec) return fail(HL_EINVAL, "batch not created");
  HIPCHK(hipGraphLaunch(B->exec, (hipStream_t)stream));
  return HL_OK;
}

extern "C" hl_status hl_batch_results(hl_batch* B, void* stream, hl_lambda_t* out, hl_status* status) {
  if (!B || !out || !status) return fail(HL_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  hl_status first = HL_OK;
  for (size_t i = 0; i < B->inst.size(); ++i) {
    const Inst& I = B->inst[i];
    unsigned long long v = 0;
    HIPCHK(hipMemcpy(&v, I.st, 8, hipMemcpyDeviceToHost));
    memset(&out[i], 0, sizeof out[i]);
    status[i] = (hl_status)(int)(v >> 32);
    if (status[i] != HL_OK) {
      if (first == HL_OK) first = status[i];
      continue;
    }
    int64_t bexp = 0;
    HIPCHK(hipMemcpy(&bexp, I.in.blk_exp, 8, hipMemcpyDeviceToHost));
    hl_status s = read_lambda(I.dm, I.base + I.L.eig, bexp, nullptr, nullptr, &out[i]);
    if (s != HL_OK) return s;
  }
  if (first != HL_OK) return fail(first, "an instance of the batch failed (see per-instance status)");
  return HL_OK;
}

extern "C" hl_status hl_batch_destroy(hl_batch* B) {
  if (!B) return HL_OK;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  delete B;
  return HL_OK;
}

// Autotuner: times the first `panels` panel steps of the factorisation under
// each candidate tuning (each replayed `reps` times after one warm-up) and
// returns the fastest.  Candidates: items per SIMD in {2, 4, 8} x range cap
// in {16, 64} x VALU below {0, 4096} bits x Karatsuba by precision or not.  Results are bit-identical
// under every candidate; only the time differs.
extern "C" hl_status hl_autotune(hl_ctx* ctx, int32_t count, const hl_instance* inst, void* plan, size_t plan_bytes,
                                 int32_t panels, hl_tune_t* best, double* best_ms) {
  if (!best) return fail(HL_EINVAL, "null output");
  const int ips[] = {2, 4, 8};
  const int caps[] = {16, 64};
  const int valu[] = {0, 4096};
  const int kara[] = {0, -1};
  double bt = 1e300;
  hl_tune_t bb{4, kMaxRanges, 0, 0};
  hipStream_t st = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hl_status result = HL_OK;
  for (int a : ips)
    for (int c : caps)
      for (int v : valu)
        for (int kk : kara) {
        hl_tune_t t{a, c, v, kk};
        hl_batch B;
        hl_status s = init_batch(ctx, count, inst, &t, plan, plan_bytes, &B);
        if (s == HL_OK) s = build(&B, panels > 0 ? panels : 2);
        if (s == HL_OK) s = capture(&B);
        if (s != HL_OK) {
          result = s;
          break;
        }
        float ms = 0;
        (void)hipGraphLaunch(B.exec, st);  // warm-up
        (void)hipEventRecord(e0, st);
        const int reps = 2;
        for (int r = 0; r < reps; ++r) (void)hipGraphLaunch(B.exec, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (B.exec) (void)hipGraphExecDestroy(B.exec);
        if (B.graph) (void)hipGraphDestroy(B.graph);
        B.exec = nullptr;
        B.graph = nullptr;
        const double per = ms / reps;
        if (per < bt) {
          bt = per;
          bb = t;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  if (result != HL_OK) return result;
  *best = bb;
  if (best_ms) *best_ms = bt;
  return HL_OK;
}
