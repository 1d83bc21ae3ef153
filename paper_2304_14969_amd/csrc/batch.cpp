// Batches of independent small kets run together (the many-circuits case).
//
// All kets live in one device arena. Running a list of circuits (one per ket)
// goes pass by pass: pass p applies the p-th fused block of every circuit
// that has one, with one launch per distinct block width, so the number of
// launches grows with the depth of the circuits, not with their count. The
// work tables and block matrices of a run are uploaded once; the launches can
// be captured into a HIP graph and replayed.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "circuit.h"
#include "qs_internal.h"

namespace qs {
void* device_alloc(size_t bytes);
void device_free(void* p);
void set_last_error(const char* msg);
}  // namespace qs

namespace {

int bfail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  qs::set_last_error(buf);
  return code;
}

int berr(hipError_t e, const char* what) {
  if (e == hipSuccess) return QS_OK;
  return bfail(QS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct Launch {
  size_t item0;  // first item of this launch in the item table
  int nitems;
  uint64_t tiles;
  int k;             // block launches: block width
  bool tile = false; // a batched tile pass (items in the tile-item table)
};

}  // namespace

struct qs_batch {
  int count = 0;
  int dtype = QS_C64;
  std::vector<int> n;
  std::vector<uint64_t> off;  // amplitude offset of each ket
  uint64_t total = 0;
  void* arena = nullptr;
  uint64_t* d_offs = nullptr;
  hipStream_t stream = nullptr;
  // tables of the last prepared run
  qs::BatchItem* d_items = nullptr;
  void* d_mats = nullptr;
  bool tiles = true;                  // complex64 kets of >= 12 qubits as tile passes
  qs::TileItem* d_titems = nullptr;   // tile items of every pass launch
  // what the prepared tables were built from: the circuits, their generations,
  // kmax and the tile switch (a run with the same reuses them)
  std::vector<std::pair<const qs_circuit*, uint64_t>> built_from;
  int built_kmax = 0;
  bool built_tiles = false;
  void* d_tdata = nullptr;            // round table, then the embedded round matrices
  size_t tmats_off = 0;               // byte offset of the matrices in d_tdata
  std::vector<Launch> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t amp_bytes(const qs_batch* b) { return b->dtype == QS_C64 ? 8 : 16; }

void drop_run(qs_batch* b) {
  if (b->d_items || b->d_mats || b->exec) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  qs::device_free(b->d_items);
  qs::device_free(b->d_mats);
  qs::device_free(b->d_titems);
  qs::device_free(b->d_tdata);
  b->d_items = nullptr;
  b->d_mats = nullptr;
  b->d_titems = nullptr;
  b->d_tdata = nullptr;
  b->launches.clear();
  b->built_from.clear();
}

// Tile passes for the kets that take them: one launch per pass index over
// every ket that has that pass. Fills use_tile; false if nothing to do.
int prepare_tiles(qs_batch* b, qs_circuit* const* circs, std::vector<char>* use_tile) {
  use_tile->assign(b->count, 0);
  if (!b->tiles || b->dtype != QS_C64) return QS_OK;
  constexpr int C = qs::kBatchTileLow, H = qs::kTileRowBits;
  std::vector<const qs::TilePlan*> plans(b->count, nullptr);
  size_t maxp = 0;
  for (int i = 0; i < b->count; ++i) {
    qs_circuit* c = circs[i];
    if (b->n[i] < C + H || c->gates.empty()) continue;
    if (!c->bplan_ok || c->bplan.C != C) {
      c->bplan = qs::plan_tiles(c->gates, b->n[i], C, H, 4, true);
      c->bplan_ok = true;
    }
    plans[i] = &c->bplan;
    bool ok = true;
    for (const auto& st : plans[i]->steps) ok = ok && !st.block;
    if (!ok) continue;
    (*use_tile)[i] = 1;
    maxp = std::max(maxp, plans[i]->steps.size());
  }
  if (!maxp) return QS_OK;
  // rounds of every ket, in ket order; round_base[i] = first round of ket i
  std::vector<int32_t> rtab;
  std::vector<float> emb;
  std::vector<int> round_base(b->count, 0);
  int nround = 0;
  for (int i = 0; i < b->count; ++i) {
    if (!(*use_tile)[i]) continue;
    round_base[i] = nround;
    for (const auto& r : plans[i]->rounds) {
      rtab.push_back(r.bits[0] | (r.bits[1] << 8) | (r.bits[2] << 16) | (r.bits[3] << 24));
      rtab.push_back(nround * qs::kRoundOperands);
      rtab.push_back(0);
      rtab.push_back(0);
      emb.resize(size_t(nround + 1) * qs::kRoundOperands);
      qs::embed_round(plans[i]->mats.data() + r.mat,
                      emb.data() + size_t(nround) * qs::kRoundOperands);
      ++nround;
    }
  }
  std::vector<qs::TileItem> items;
  for (size_t p = 0; p < maxp; ++p) {
    Launch L{items.size(), 0, 0, 0, true};
    for (int i = 0; i < b->count; ++i) {
      if (!(*use_tile)[i] || p >= plans[i]->steps.size()) continue;
      const qs::TileStep& st = plans[i]->steps[p];
      qs::TileItem it{};
      it.amp_off = b->off[i];
      it.first_tile = L.tiles;
      for (int j = 0; j < H; ++j) it.rows.b[j] = st.hb[j];
      it.r0 = round_base[i] + st.r0;
      it.nr = st.nr;
      items.push_back(it);
      L.tiles += uint64_t(1) << (b->n[i] - C - H);
      ++L.nitems;
    }
    if (L.nitems) b->launches.push_back(L);
  }
  const size_t rbytes = (rtab.size() * sizeof(int32_t) + 255) / 256 * 256;
  b->tmats_off = rbytes;
  b->d_titems = static_cast<qs::TileItem*>(qs::device_alloc(items.size() * sizeof(qs::TileItem)));
  b->d_tdata = qs::device_alloc(rbytes + emb.size() * sizeof(float));
  if (!b->d_titems || !b->d_tdata) return bfail(QS_E_NOMEM, "batch tile tables");
  std::vector<unsigned char> host(rbytes + emb.size() * sizeof(float), 0);
  std::memcpy(host.data(), rtab.data(), rtab.size() * sizeof(int32_t));
  std::memcpy(host.data() + rbytes, emb.data(), emb.size() * sizeof(float));
  hipError_t e = hipMemcpy(b->d_titems, items.data(), items.size() * sizeof(qs::TileItem),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_tdata, host.data(), host.size(), hipMemcpyHostToDevice);
  return berr(e, "batch tile table upload");
}

// Builds and uploads the pass tables of a run (synchronous upload), unless
// the tables in place were built from the same, unchanged circuits.
int prepare(qs_batch* b, qs_circuit* const* circs, int kmax) {
  if (!b->built_from.empty() && b->built_kmax == kmax && b->built_tiles == b->tiles &&
      !b->exec) {
    bool same = true;
    for (int i = 0; i < b->count && same; ++i)
      same = circs[i] == b->built_from[i].first &&
             circs[i]->generation == b->built_from[i].second;
    if (same) return QS_OK;
  }
  for (int i = 0; i < b->count; ++i) {
    qs_circuit* c = circs[i];
    if (!c) return bfail(QS_E_INVAL, "circuit %d is NULL", i);
    if (c->n != b->n[i]) return bfail(QS_E_INVAL, "circuit %d has %d qubits, ket %d", i, c->n, b->n[i]);
    for (int q = 0; q < c->n; ++q)
      if (c->pos[q] != q) return bfail(QS_E_UNSUPPORTED, "batched circuits cannot contain SWAP gates");
    if (!c->planned || c->kmax != kmax)
      if (int rc = qs::circuit_plan_blocks(c, kmax)) return rc;
    for (const auto& blk : c->blocks)
      if (blk.k > 5) return bfail(QS_E_UNSUPPORTED, "batched blocks have at most 5 qubits");
  }
  drop_run(b);
  std::vector<char> use_tile;
  if (int rc = prepare_tiles(b, circs, &use_tile)) {
    drop_run(b);
    return rc;
  }
  // matrices: every block of every circuit that runs as blocks
  std::vector<std::vector<uint64_t>> moff(b->count);
  uint64_t mtotal = 0;
  size_t maxblocks = 0;
  for (int i = 0; i < b->count; ++i) {
    if (use_tile[i]) continue;
    for (const auto& blk : circs[i]->blocks) {
      moff[i].push_back(mtotal);
      mtotal += blk.m.size();
    }
    maxblocks = std::max(maxblocks, circs[i]->blocks.size());
  }
  std::vector<qs::BatchItem> items;
  for (size_t p = 0; p < maxblocks; ++p) {
    for (int k = 1; k <= 5; ++k) {
      Launch L{items.size(), 0, 0, k};
      for (int i = 0; i < b->count; ++i) {
        if (use_tile[i]) continue;
        const auto& blocks = circs[i]->blocks;
        if (p >= blocks.size() || blocks[p].k != k) continue;
        qs::BatchItem it{};
        it.amp_off = b->off[i];
        it.first_tile = L.tiles;
        it.mat_off = moff[i][p];
        it.n = b->n[i];
        it.k = k;
        int s[5];
        for (int j = 0; j < k; ++j) s[j] = it.q[j] = blocks[p].q[j];
        std::sort(s, s + k);
        for (int j = 0; j < k; ++j) it.sorted[j] = s[j];
        const uint64_t groups = uint64_t(1) << (b->n[i] - k);
        L.tiles += (groups + 255) / 256;
        items.push_back(it);
        ++L.nitems;
      }
      if (L.nitems) b->launches.push_back(L);
    }
  }
  const size_t esz = b->dtype == QS_C64 ? sizeof(float) : sizeof(double);
  b->d_items = static_cast<qs::BatchItem*>(qs::device_alloc(std::max<size_t>(1, items.size()) * sizeof(qs::BatchItem)));
  b->d_mats = qs::device_alloc(std::max<uint64_t>(1, 2 * mtotal) * esz);
  if (!b->d_items || !b->d_mats) {
    drop_run(b);
    return bfail(QS_E_NOMEM, "batch tables");
  }
  hipError_t e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(qs::BatchItem),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    if (b->dtype == QS_C64) {
      std::vector<float> h(2 * mtotal);
      for (int i = 0; i < b->count; ++i)
        for (size_t p = 0; !use_tile[i] && p < circs[i]->blocks.size(); ++p) {
          const auto& m = circs[i]->blocks[p].m;
          for (size_t j = 0; j < m.size(); ++j) {
            h[2 * (moff[i][p] + j)] = float(m[j].real());
            h[2 * (moff[i][p] + j) + 1] = float(m[j].imag());
          }
        }
      e = hipMemcpy(b->d_mats, h.data(), h.size() * esz, hipMemcpyHostToDevice);
    } else {
      std::vector<double> h(2 * mtotal);
      for (int i = 0; i < b->count; ++i)
        for (size_t p = 0; !use_tile[i] && p < circs[i]->blocks.size(); ++p) {
          const auto& m = circs[i]->blocks[p].m;
          for (size_t j = 0; j < m.size(); ++j) {
            h[2 * (moff[i][p] + j)] = m[j].real();
            h[2 * (moff[i][p] + j) + 1] = m[j].imag();
          }
        }
      e = hipMemcpy(b->d_mats, h.data(), h.size() * esz, hipMemcpyHostToDevice);
    }
  }
  if (e != hipSuccess) {
    drop_run(b);
    return berr(e, "batch table upload");
  }
  b->built_from.clear();
  for (int i = 0; i < b->count; ++i) b->built_from.emplace_back(circs[i], circs[i]->generation);
  b->built_kmax = kmax;
  b->built_tiles = b->tiles;
  return QS_OK;
}

hipError_t enqueue(qs_batch* b) {
  for (const Launch& L : b->launches) {
    if (L.tile) {
      const hipError_t e = qs::launch_tile_mfma_batch(
          static_cast<float*>(b->arena), b->d_titems + L.item0, L.nitems, L.tiles, b->d_tdata,
          reinterpret_cast<const float*>(static_cast<const char*>(b->d_tdata) + b->tmats_off),
          b->stream);
      if (e != hipSuccess) return e;
      continue;
    }
    hipError_t e =
        b->dtype == QS_C64
            ? qs::launch_batch_fused(static_cast<float*>(b->arena), b->d_items + L.item0, L.nitems,
                                     L.tiles, L.k, static_cast<const float*>(b->d_mats), b->stream)
            : qs::launch_batch_fused(static_cast<double*>(b->arena), b->d_items + L.item0, L.nitems,
                                     L.tiles, L.k, static_cast<const double*>(b->d_mats), b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int qs_batch_create(int count, const int* n_each, int dtype, qs_batch** out) {
  if (!out || !n_each) return bfail(QS_E_INVAL, "NULL argument");
  if (count < 1) return bfail(QS_E_INVAL, "count = %d", count);
  if (dtype != QS_C64 && dtype != QS_C128) return bfail(QS_E_INVAL, "unknown dtype %d", dtype);
  qs_batch* b = new qs_batch();
  b->count = count;
  b->dtype = dtype;
  for (int i = 0; i < count; ++i) {
    if (n_each[i] < 1 || n_each[i] > 30) {
      delete b;
      return bfail(QS_E_INVAL, "ket %d: n = %d outside [1, 30]", i, n_each[i]);
    }
    b->n.push_back(n_each[i]);
    b->off.push_back(b->total);
    // 64-amplitude alignment keeps every ket on whole cache lines
    b->total += ((uint64_t(1) << n_each[i]) + 63) / 64 * 64;
  }
  b->arena = qs::device_alloc(b->total * amp_bytes(b));
  b->d_offs = static_cast<uint64_t*>(qs::device_alloc(count * sizeof(uint64_t)));
  if (!b->arena || !b->d_offs) {
    qs::device_free(b->arena);
    qs::device_free(b->d_offs);
    delete b;
    return bfail(QS_E_NOMEM, "batch arena of %llu amplitudes", (unsigned long long)b->total);
  }
  hipError_t e = hipMemcpy(b->d_offs, b->off.data(), count * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = b->dtype == QS_C64
            ? qs::launch_batch_reset(static_cast<float*>(b->arena), b->total, b->d_offs, count, b->stream)
            : qs::launch_batch_reset(static_cast<double*>(b->arena), b->total, b->d_offs, count, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    qs::device_free(b->arena);
    qs::device_free(b->d_offs);
    delete b;
    return berr(e, "batch init");
  }
  *out = b;
  return QS_OK;
}

int qs_batch_free(qs_batch* b) {
  if (!b) return QS_OK;
  drop_run(b);
  (void)hipStreamSynchronize(b->stream);
  qs::device_free(b->arena);
  qs::device_free(b->d_offs);
  delete b;
  return QS_OK;
}

int qs_batch_set_stream(qs_batch* b, void* stream) {
  if (!b) return bfail(QS_E_INVAL, "batch is NULL");
  b->stream = static_cast<hipStream_t>(stream);
  return QS_OK;
}

int qs_batch_reset(qs_batch* b) {
  if (!b) return bfail(QS_E_INVAL, "batch is NULL");
  hipError_t e = b->dtype == QS_C64
                     ? qs::launch_batch_reset(static_cast<float*>(b->arena), b->total, b->d_offs, b->count, b->stream)
                     : qs::launch_batch_reset(static_cast<double*>(b->arena), b->total, b->d_offs, b->count, b->stream);
  return berr(e, "batch reset");
}

int qs_batch_run(qs_batch* b, qs_circuit* const* circuits, int kmax) {
  if (!b || !circuits) return bfail(QS_E_INVAL, "NULL argument");
  if (kmax == 0) kmax = 4;
  if (kmax < 1 || kmax > 5) return bfail(QS_E_INVAL, "kmax = %d outside [1, 5]", kmax);
  if (int rc = prepare(b, circuits, kmax)) return rc;
  return berr(enqueue(b), "batch run");
}

int qs_batch_capture(qs_batch* b, qs_circuit* const* circuits, int kmax) {
  if (!b || !circuits) return bfail(QS_E_INVAL, "NULL argument");
  if (!b->stream) return bfail(QS_E_INVAL, "graph capture needs a non-default stream");
  if (kmax == 0) kmax = 4;
  if (kmax < 1 || kmax > 5) return bfail(QS_E_INVAL, "kmax = %d outside [1, 5]", kmax);
  if (int rc = prepare(b, circuits, kmax)) return rc;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return berr(e, "begin capture");
  hipError_t le = enqueue(b);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->stream, &g);
  if (le != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return berr(le != hipSuccess ? le : e, "capture");
  }
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->graph = nullptr;
    b->exec = nullptr;
    return berr(e, "graph instantiate");
  }
  return QS_OK;
}

int qs_batch_replay(qs_batch* b) {
  if (!b) return bfail(QS_E_INVAL, "batch is NULL");
  if (!b->exec) return bfail(QS_E_INVAL, "no captured run");
  return berr(hipGraphLaunch(b->exec, b->stream), "graph launch");
}

int qs_batch_use_tiles(qs_batch* b, int on) {
  if (!b) return bfail(QS_E_INVAL, "batch is NULL");
  drop_run(b);
  b->tiles = on != 0;
  return QS_OK;
}

int qs_batch_info(const qs_batch* b, int* launches, uint64_t* total_amps) {
  if (!b) return bfail(QS_E_INVAL, "batch is NULL");
  if (launches) *launches = int(b->launches.size());
  if (total_amps) *total_amps = b->total;
  return QS_OK;
}

int qs_batch_amplitudes(qs_batch* b, int i, void* host_out, uint64_t count, int out_dtype) {
  if (!b || !host_out) return bfail(QS_E_INVAL, "NULL argument");
  if (i < 0 || i >= b->count) return bfail(QS_E_INVAL, "ket %d out of range", i);
  if (count != (uint64_t(1) << b->n[i])) return bfail(QS_E_INVAL, "count != 2^%d", b->n[i]);
  if (out_dtype != b->dtype) return bfail(QS_E_UNSUPPORTED, "batch readout keeps the ket's precision");
  hipError_t e = hipMemcpyAsync(host_out, static_cast<const char*>(b->arena) + b->off[i] * amp_bytes(b),
                                count * amp_bytes(b), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return berr(e, "batch readout");
}

int qs_batch_synchronize(qs_batch* b) {
  if (!b) return bfail(QS_E_INVAL, "batch is NULL");
  return berr(hipStreamSynchronize(b->stream), "batch synchronize");
}

}  // extern "C"
