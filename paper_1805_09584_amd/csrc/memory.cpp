// Device storage of a context.
//
// Every lattice-sized buffer of the library (repacked links, Krylov vectors,
// multigrid data, network buffers) is taken through dev_alloc / dev_free.  Two
// modes:
//  * managed (default): each buffer is its own hipMalloc, freed by dev_free or
//    ndtm_destroy;
//  * caller workspace (ndtm_set_workspace): buffers are carved out of one
//    device region the caller owns, first fit over a free list ordered by
//    offset, neighbouring free blocks merged on release.  No hipMalloc or
//    hipFree happens in this mode; a request the region cannot hold fails and
//    the calling entry point returns NDTM_ENOMEM.
// Both modes count the live and peak bytes and the device allocations made,
// which ndtm_workspace_stats reports.
#include <algorithm>
#include <map>

#include "ctx.h"
#include "mlp.h"

namespace ndtm {

constexpr size_t kAlign = 256;

static size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
  std::map<size_t, size_t> free_;  // offset -> size, disjoint, sorted
};

void* dev_alloc(ndtm_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 1;
  const size_t n = round_up(bytes);
  void* p = nullptr;
  if (c->arena) {
    Arena* A = c->arena;
    for (auto it = A->free_.begin(); it != A->free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, rest = it->second - n;
      A->free_.erase(it);
      if (rest) A->free_[off + n] = rest;
      p = A->base + off;
      break;
    }
    if (!p) return nullptr;
  } else {
    if (hipMalloc(&p, n) != hipSuccess) return nullptr;
    ++c->mem_device_allocs;
  }
  c->mem_sizes[p] = n;
  c->mem_live += n;
  c->mem_peak = std::max(c->mem_peak, c->mem_live);
  return p;
}

void dev_free(ndtm_ctx* c, void* p) {
  if (!p) return;
  auto s = c->mem_sizes.find(p);
  if (s == c->mem_sizes.end()) return;
  const size_t n = s->second;
  c->mem_sizes.erase(s);
  c->mem_live -= n;
  if (!c->arena) {
    (void)hipFree(p);
    return;
  }
  Arena* A = c->arena;
  size_t off = static_cast<char*>(p) - A->base, len = n;
  auto next = A->free_.lower_bound(off);
  if (next != A->free_.end() && off + len == next->first) {
    len += next->second;
    next = A->free_.erase(next);
  }
  if (next != A->free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      return;
    }
  }
  A->free_[off] = len;
}

size_t dev_largest_free(const ndtm_ctx* c) {
  if (c->arena) {
    size_t m = 0;
    for (const auto& f : c->arena->free_) m = std::max(m, f.second);
    return m;
  }
  size_t fr = 0, tot = 0;
  (void)hipMemGetInfo(&fr, &tot);
  return fr;
}

void arena_release(ndtm_ctx* c) {
  delete c->arena;
  c->arena = nullptr;
}

int arena_set(ndtm_ctx* c, void* dev, size_t bytes) {
  if (!c->mem_sizes.empty())
    return fail(c, NDTM_ESTATE, "set_workspace: call it before set_gauge, while the context holds no lattice storage");
  arena_release(c);
  if (!dev) return NDTM_OK;  // back to managed storage
  if (reinterpret_cast<uintptr_t>(dev) % kAlign)
    return fail(c, NDTM_EINVAL, "set_workspace: the region must be 256-byte aligned");
  if (bytes < kAlign) return fail(c, NDTM_EINVAL, "set_workspace: region too small");
  Arena* A = new Arena();
  A->base = static_cast<char*>(dev);
  A->bytes = bytes / kAlign * kAlign;
  A->free_[0] = A->bytes;
  c->arena = A;
  return NDTM_OK;
}

}  // namespace ndtm

using namespace ndtm;

namespace {

size_t R(size_t b) { return round_up(b); }

struct Sizes {
  const ndtm_ctx* c;
  size_t n, stride;
  size_t half(int prec) const {
    if (prec == P64) return R(n * 16);
    if (prec == P32) return R(n * 8);
    return R(n * 4) + R(stride * 4);  // FP16 values and one FP32 scale per site
  }
  size_t full(int prec) const { return R(2 * n * (prec == P64 ? 16 : 8)); }
};

}  // namespace

extern "C" {

int ndtm_set_workspace(ndtm_ctx* c, void* dev, size_t bytes) {
  if (!c) return NDTM_EINVAL;
  return arena_set(c, dev, bytes);
}

int ndtm_trim(ndtm_ctx* c) {
  if (!c) return NDTM_EINVAL;
  NDTM_HIP(c, hipSetDevice(c->device));
  NDTM_HIP(c, hipDeviceSynchronize());
  // the multigrid cycle's fields (mg_*) belong to the setup: captured cycle graphs use them
  for (auto it = c->bufs.begin(); it != c->bufs.end();) {
    if (it->first.compare(0, 3, "mg_") != 0) {
      dev_free(c, it->second.p);
      it = c->bufs.erase(it);
    } else {
      ++it;
    }
  }
  return NDTM_OK;
}

int ndtm_workspace_stats(const ndtm_ctx* c, size_t* live, size_t* peak, long long* device_allocs) {
  if (!c) return NDTM_EINVAL;
  if (live) *live = c->mem_live;
  if (peak) *peak = c->mem_peak;
  if (device_allocs) *device_allocs = c->mem_device_allocs;
  return NDTM_OK;
}

int ndtm_workspace_bytes(const ndtm_ctx* c, int n_shifts, const ndtm_mg_params* mg, const ndtm_solve_params* sp,
                         size_t* bytes) {
  if (!c || !bytes) return NDTM_EINVAL;
  if (sp && (n_shifts < 1 || n_shifts > NDTM_MAX_SHIFTS)) return NDTM_EINVAL;
  const Sizes z{c, half_elems(c), (size_t)c->g.stride};
  size_t t = 0;
  // links: FP64, FP32 and FP16 copies of both parities
  for (size_t es : {16, 8, 4}) t += 2 * R(36 * z.stride * es);
  // FP64 SU(3) links in eight parameters (four complex words per link and direction)
  t += 2 * R(16 * z.stride * 16);
  // clover site blocks (with c_sw set): a + C on both parities and the even inverse, FP64 and FP32
  if (c->csw != 0.0)
    for (size_t es : {8, 4}) t += 2 * R(72 * z.stride * es) + R(144 * z.stride * es) + (es == 8 ? R(256) : 0);
  // ndtm_apply in each precision: x, y, the even intermediate, Q x and the even output
  for (int prec : {P64, P32, P16}) t += 5 * z.half(prec);
  if (sp) {
    const int nsh = n_shifts;
    const int n_mms = std::max(1, std::min(sp->n_mmscg, nsh));
    const bool mg_phase = n_mms < nsh;
    const size_t h64 = z.half(P64);
    t += (size_t)(1 + nsh) * h64;  // b and the solutions
    t += 5 * h64;                  // true residual, its Q^2 temporaries, CG polish
    t += 6 * h64;                  // base Krylov vectors and the first shifted direction
    t += (size_t)nsh * h64;        // solutions of ndtm_solve_rational
    const size_t mg_fields = mg_phase ? (size_t)mg_region_fields(sp->fgmres_restart, mg && mg->pair_signs) : 0;
    {
      const int n_pred = mg_phase ? std::max(0, std::min(sp->mms_predict, nsh - n_mms)) : 0;
      int defer = std::min(sp->mms_defer, kMaxDefer);
      if (defer < 2) defer = 0;
      const size_t mms_fields = (size_t)(n_mms + n_pred - 1 + defer);
      t += R(std::max(mg_fields, mms_fields) * z.n * 16);
      if (n_pred > 0) t += 2 * h64;
      // mixed form: the stencil's operands (p, w and two temporaries) in FP32 and FP16
      if (sp->precision == NDTM_PREC_F16 && defer) t += 4 * z.half(P32) + 4 * z.half(P16);
    }
    if (mg_phase) {
      t += 2 * h64;  // guess: projection or network sample vectors
      if (sp->guess == NDTM_GUESS_MLP)
        t += 4 * R(kMlpNParam * 4) + R(kMlpNParam * 2) +
             R(kMlpNFeat * 4) + 4 * R(kMlpKMax * 4) + R(kMlpKMax * kMlpKMax * 4) + R(4) + R(kMlpNParam * 4);
    }
  }
  if (mg) {
    const int dims[4] = {c->g.T, c->g.Lz, c->g.Ly, c->g.Lx};
    size_t nloc = 1;
    for (int i = 0; i < 4; ++i) {
      if (mg->block[i] < 1 || dims[i] % mg->block[i]) return NDTM_EINVAL;
      nloc *= (size_t)mg->block[i];
    }
    if (mg->n_vec < 2 || mg->n_vec > 32 || mg->coarse_iters < 1 || mg->coarse_iters > 32) return NDTM_EINVAL;
    const size_t Vc = (size_t)c->V / nloc, Nv = (size_t)mg->n_vec, n2 = 2 * Nv, kc = (size_t)mg->coarse_iters;
    const int cp = mg->precision == NDTM_PREC_F64 ? P64 : P32;
    const bool f16 = mg->precision == NDTM_PREC_F16;
    const size_t cs = cp == P64 ? 16 : 8;
    const size_t nP = Vc * nloc * 12 * Nv, nD = Vc * 5 * n2 * n2, nB = Vc * 2 * Nv * Nv, nc = Vc * 2 * n2;
    t += R(nP * 16) + R(nD * 16) + R(nB * 16);
    // cycle copies: P in FP32, or in FP16 with one scale per fine site
    if (cp == P32) t += R(nP * (f16 ? 4 : 8)) + R(nD * 8) + R(nB * 8) + (f16 ? R(Vc * nloc * 4) : 0);
    t += (kc + 1 + 5) * R(nc * cs) + 2 * R(2 * (kc + 1) * (kc + 1) * 8) + R((kc + 1) * 8) + R(2 * (kc + 1) * 8) +
         R(64) + R(128) + R(6 * (size_t)hop_grid(c->g) * 8);
    t += 4 * z.full(cp);  // cycle vectors
    // paired signs: the second system's cycle vectors and the FP64 coarse pair
    if (mg->pair_signs) t += 2 * z.full(cp) + 2 * R(2 * nc * 16);
    // setup temporaries: partial self blocks, test vectors and the inverse-iteration CG
    t += R(Vc * 8 * n2 * n2 * 16) + ((Nv + 1) / 2 + 6) * z.full(P64) + 2 * z.full(cp);
    if (mg->setup_prec == NDTM_PREC_F32) t += 5 * z.full(P32);  // the FP32 inverse iteration's CG vectors
    // the multigrid calls of the ABI: a full FP64 field and two in the cycle precision, the
    // batched coarse solve of 8 systems
    const size_t per = 2 * (2 * (kc + 1) * (kc + 1)) + 3 * (kc + 1) + 2;
    t += z.full(P64) + 2 * z.full(cp) + R((kc + 1) * 8 * nc * 16) + 2 * R(8 * nc * 16) + R(8 * per * 8) +
         R(8 * (8 + 2 * (kc + 1) * 256) * 8);
  }
  // first-fit slack: two half fields
  t += 2 * z.half(P64);
  *bytes = t;
  return NDTM_OK;
}

}  // extern "C"
