// Serving: continuous batching of independent compress requests.
//
// Admission.  A request (one image, its own transform, n, r, qstep, dtype) is
// charged its input plus its outputs against the HBM budget and reserves its
// outputs in the server's arena, a ring: batches complete in submission
// order, so space is released oldest first.  adct_server_submit does this on
// the host only.
//
// Batches.  adct_server_flush takes the queued requests (oldest first) into a
// free batch slot.  Each slot has its own stream, ordered after the caller's
// stream, on which it issues: the request tables (pinned host -> device), a
// clear of the per-request error energies, one launch per class (transform,
// n, dtype, quantiser, r bound) covering all of that class's requests, the
// copy of the error energies back to pinned host memory, the optional host
// copies of outputs, and the slot's completion event.  Requests that arrive
// while batches run wait in the queue and form the next batch, which runs
// on another slot's stream beside the batches still on the device: the
// batch size follows the load and consecutive batches overlap.  Batches may
// therefore complete out of order; an arena block is reused once every
// older block has been released.
//
// Class launches.  Workgroup i of a class launch processes one tile group
// (64 8x8 tiles, or 256/n tiles of size n) of one request.  The request is
// found from the first-item offsets of the class's requests with two
// wave-wide ballots, then the same fused code as the plain kernels runs on
// that group.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/adct.h"
#include "jam_group.hpp"
#include "tile8.hpp"

namespace adct {

// defined in api.hip
int set_error(int status, const char* msg);
int build_tables_for(int kind, int n, int qstep, Tables* out);

namespace {

// Device record of one request of a class launch.
struct SReq {
  const void* src;
  void* dst;
  int32_t* kept;
  float* scaled;                // nullable
  unsigned long long* sse;
  int64_t pitch;                // pixels, source and reconstruction
  int32_t tiles_x;
  int32_t groups_x;             // tile groups per tile row
  int32_t r;
  int32_t pad;
  Tables t;
};

constexpr int kMaxBatch = 4096;   // requests per batch (and per class launch)

// Index q of the request that owns workgroup `item`: the last q with
// begins[q] <= item (begins[0] = 0, increasing).  A ballot over every 64th
// request picks the segment, a second ballot the request inside it.  Every
// lane of the wave calls it; n_req <= 4096.
__device__ __forceinline__ int find_request(const int* begins, int n_req, int item) {
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (n_req > 64) {
    const int q = lane * 64;
    const bool le = q < n_req && begins[q] <= item;
    base = (__popcll(__ballot(le)) - 1) * 64;
  }
  const int q = base + lane;
  const bool le = q < n_req && begins[q] <= item;
  return base + __popcll(__ballot(le)) - 1;
}

template <int KIND, int DT, int RB, bool QUANT>
__global__ __launch_bounds__(t8::kWave) void serve8(const SReq* reqs, const int* begins,
                                                    int n_req) {
  __shared__ int lds[t8::kWave * t8::row_stride(RB)];
  const int item = blockIdx.x;
  const int q = find_request(begins, n_req, item);
  const SReq& rq = reqs[q];
  const int local = item - begins[q];
  const int ty = local / rq.groups_x;
  const int tx0 = (local - ty * rq.groups_x) * t8::kWave;
  const int lane = threadIdx.x;
  t8::WaveIO io;
  io.src = rq.src;
  io.dst = rq.dst;
  io.pitch = rq.pitch;
  io.tile_pix = static_cast<int64_t>(ty) * 8 * rq.pitch + static_cast<int64_t>(tx0 + lane) * 8;
  io.lane = lane;
  io.nact = min(t8::kWave, rq.tiles_x - tx0);
  io.active = lane < io.nact;
  io.r = rq.r;
  const int64_t tile0 = static_cast<int64_t>(ty) * rq.tiles_x + tx0;
  io.kept = rq.kept + tile0 * rq.r;
  io.scaled = rq.scaled != nullptr ? rq.scaled + tile0 * rq.r : nullptr;
  io.sse = true;
  const unsigned long long e =
      t8::compress_wave<KIND, DT, RB, QUANT, true, false>(lds, rq.t, io);
  block_add_sse<t8::kWave>(rq.sse, e, nullptr);
}

// KB: compile-time kept bound of the class (4, 8 or N; zonal r <= KB (KB + 1) / 2).
template <int KIND, int N, int DT, bool QUANT, int KB>
__global__ __launch_bounds__(jam::kBlock) void serve_jam(const SReq* reqs, const int* begins,
                                                         int n_req) {
  using C = jam::Cfg<N, jam::kBlock, KB>;
  __shared__ int S[C::WORDS];
  __shared__ jam::Shared<N> sh;
  __shared__ unsigned long long red[jam::kBlock / 64];
  const int item = blockIdx.x;
  const int q = find_request(begins, n_req, item);
  const SReq& rq = reqs[q];
  jam::load_tables<KIND, N, jam::kBlock, KB>(sh, rq.t, rq.r);
  const int local = item - begins[q];
  const int ty = local / rq.groups_x;
  const int tx0 = (local - ty * rq.groups_x) * C::TPW;
  const int k = threadIdx.x % C::TPW;
  jam::GroupIO io;
  io.src = rq.src;
  io.dst = rq.dst;
  io.pitch = rq.pitch;
  io.tile_pix = static_cast<int64_t>(ty) * N * rq.pitch + static_cast<int64_t>(tx0 + k) * N;
  io.nact = min(C::TPW, rq.tiles_x - tx0);
  io.active = k < io.nact;
  io.r = rq.r;
  const int64_t tile0 = static_cast<int64_t>(ty) * rq.tiles_x + tx0;
  io.kept = rq.kept + tile0 * rq.r;
  io.scaled = rq.scaled != nullptr ? rq.scaled + tile0 * rq.r : nullptr;
  io.sse = true;
  const unsigned long long e =
      jam::compress_group<KIND, N, DT, QUANT, jam::kBlock, false, KB>(S, sh, io);
  block_add_sse<jam::kBlock>(rq.sse, e, red);
}

// ------------------------------------------------------------- host side
// Class of a request: requests of one class share one kernel.
struct ClassKey {
  int n, kind, dtype, quant, rb;
  bool operator<(const ClassKey& o) const {
    return std::tie(n, kind, dtype, quant, rb) < std::tie(o.n, o.kind, o.dtype, o.quant, o.rb);
  }
  bool operator!=(const ClassKey& o) const { return o < *this || *this < o; }
};

// Compile-time bound of the kernel used for a request.  8x8: a bound on r
// (the arithmetic that only feeds zig-zag positions >= RB is dropped).
// 16x16 / 32x32: the kept bound KB, every kept coefficient having v, u < KB
// (4 for zonal r <= 10, 8 for r <= 36: the zig-zag prefixes of 4 and 8
// anti-diagonals), which prunes the butterflies and the LDS exchanges.
int rb_of(int n, int r, int qstep) {
  if (n != 8) return qstep > 0 ? n : (r <= 10 ? 4 : (r <= 36 ? 8 : n));
  if (qstep > 0) return 64;
  return r <= 10 ? 10 : (r <= 28 ? 28 : 64);
}

ClassKey class_of(const adct_request_t& q) {
  return ClassKey{q.n, q.transform, q.dtype, q.qstep > 0 ? 1 : 0, rb_of(q.n, q.r, q.qstep)};
}

int groups_x_of(int n, int tiles_x) {
  const int per = n == 8 ? t8::kWave : jam::kBlock / n;
  return (tiles_x + per - 1) / per;
}

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct Member {
  adct_request_t req;
  int64_t charge = 0;     // budget bytes (input + outputs)
  int64_t seq = 0;        // arena block: allocation number, offset, length
  int64_t off = 0;
  int64_t len = 0;
  int64_t recon_off = 0, kept_off = 0, scaled_off = -1;
  int table = 0;          // index in the batch's request table
};

// A batch's table travels as one block, in pinned host memory and on the
// device: m request records, m first-item offsets, m error energies (zeros
// on upload, so no fill kernel is needed), each part 16-byte aligned.
struct TableLayout {
  size_t begins, sse, bytes;
};

inline size_t align16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

inline TableLayout table_layout(size_t m) {
  TableLayout l;
  l.begins = align16(m * sizeof(SReq));
  l.sse = align16(l.begins + m * sizeof(int));
  l.bytes = l.sse + m * sizeof(unsigned long long);
  return l;
}

struct Slot {
  char* d_table = nullptr;       // device copy of the batch table
  char* h_table = nullptr;       // pinned host staging of the batch table
  unsigned long long* h_sse = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;    // recorded on the caller's stream at flush
  hipEvent_t done = nullptr;
  std::vector<Member> members;   // submission order
  int64_t id = -1;
  double launch_ms = 0.0;        // server clock at the flush that launched it
};

struct Block {
  int64_t off, len;
  bool freed;
};

int hip_fail(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof(buf), "server: %s: %s", what, hipGetErrorString(e));
  return set_error(ADCT_E_HIP, buf);
}

}  // namespace
}  // namespace adct

using namespace adct;

struct adct_server {
  int64_t budget = 0;
  int max_inflight = 1;
  int max_batch = 1;
  hipStream_t stream = nullptr;
  std::chrono::steady_clock::time_point t0;
  // arena ring: blocks in allocation order; block seq is live[seq - seq_front]
  char* arena = nullptr;
  std::deque<Block> live;
  int64_t seq_front = 0;
  int64_t charged = 0;
  std::deque<Member> queue;
  std::vector<Slot> slots;
  std::vector<int> inflight;      // slot indices, launch order
  std::vector<int> free_slots;
  std::vector<Member> to_release; // reported by the last poll
  int64_t next_batch = 0;
  hipEvent_t origin = nullptr;
  double origin_ms = 0.0;
  bool device_ready = false;
  std::map<std::tuple<int, int, int>, Tables> tables;
  int64_t n_submitted = 0, n_completed = 0, n_refused = 0, max_seen = 0;

  double clock_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }

  // Reserve len bytes after the newest block, wrapping to offset 0 when the
  // end of the arena is reached; space is free up to the oldest live block.
  bool ring_alloc(int64_t len, int64_t* off, int64_t* seq) {
    if (len > budget) return false;
    if (live.empty()) {
      *off = 0;
    } else {
      const int64_t oldest = live.front().off;
      const int64_t end = live.back().off + live.back().len;
      const bool wrapped = live.back().off < oldest;
      if (!wrapped && end + len <= budget) *off = end;
      else if (!wrapped && len <= oldest) *off = 0;
      else if (wrapped && end + len <= oldest) *off = end;
      else return false;
    }
    *seq = seq_front + static_cast<int64_t>(live.size());
    live.push_back(Block{*off, len, false});
    return true;
  }

  void ring_release(int64_t seq) {
    live[seq - seq_front].freed = true;
    while (!live.empty() && live.front().freed) {
      live.pop_front();
      ++seq_front;
    }
  }
};

namespace {

int validate(const adct_request_t& q) {
  char msg[200];
  if (q.transform != ADCT_T1 && q.transform != ADCT_T2)
    return set_error(ADCT_E_ARG, "server: transform must be ADCT_T1 or ADCT_T2");
  if (q.n != 8 && q.n != 16 && q.n != 32) return set_error(ADCT_E_ARG, "server: n must be 8, 16 or 32");
  if (q.dtype != ADCT_U8 && q.dtype != ADCT_I16) return set_error(ADCT_E_ARG, "server: bad dtype");
  if (q.r < 1 || q.r > q.n * q.n) {
    snprintf(msg, sizeof(msg), "server: r=%d outside [1, %d]", q.r, q.n * q.n);
    return set_error(ADCT_E_ARG, msg);
  }
  if (q.qstep < 0 || q.qstep > 4096) return set_error(ADCT_E_ARG, "server: qstep outside [0, 4096]");
  if (q.height <= 0 || q.width <= 0 || q.height % q.n || q.width % q.n || q.pitch < q.width) {
    snprintf(msg, sizeof(msg), "server: %dx%d (pitch %lld) is not a multiple of n=%d", q.height,
             q.width, static_cast<long long>(q.pitch), q.n);
    return set_error(ADCT_E_SHAPE, msg);
  }
  if (q.d_src == nullptr) return set_error(ADCT_E_ARG, "server: null source");
  if (q.h_scaled != nullptr && !q.want_scaled)
    return set_error(ADCT_E_ARG, "server: h_scaled needs want_scaled");
  const int esize = q.dtype == ADCT_U8 ? 1 : 2;
  const int align = std::min(16, q.n * esize);
  if (reinterpret_cast<uintptr_t>(q.d_src) % align || (q.pitch * esize) % align)
    return set_error(ADCT_E_ALIGN, "server: source rows must be aligned to min(16, n * pixel size) bytes");
  return ADCT_OK;
}

// Outputs of a request inside its arena block and its budget charge.
void layout(Member& m) {
  const adct_request_t& q = m.req;
  const int esize = q.dtype == ADCT_U8 ? 1 : 2;
  const int64_t tiles = static_cast<int64_t>(q.height / q.n) * (q.width / q.n);
  const int64_t image = static_cast<int64_t>(q.height) * q.pitch * esize;
  m.recon_off = 0;
  m.kept_off = align256(image);
  int64_t end = m.kept_off + align256(tiles * q.r * 4);
  m.scaled_off = -1;
  if (q.want_scaled) {
    m.scaled_off = end;
    end += align256(tiles * q.r * 4);
  }
  m.len = end;
  m.charge = image + end;
}

int ensure_device(adct_server* s) {
  if (s->device_ready) return ADCT_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&s->arena), s->budget);
  if (e != hipSuccess) {
    s->arena = nullptr;
    return hip_fail(e, "arena allocation");
  }
  s->slots.resize(s->max_inflight);
  for (int i = 0; i < s->max_inflight; ++i) {
    Slot& sl = s->slots[i];
    const size_t nb = s->max_batch;
    const size_t tb = table_layout(nb).bytes;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sl.d_table), tb);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_table), tb, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_sse), nb * 8, 0);
    if (e == hipSuccess) e = hipEventCreate(&sl.done);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "batch slot allocation");
    s->free_slots.push_back(s->max_inflight - 1 - i);
  }
  // Clock alignment: the origin event's host time is taken as the moment its
  // completion is observed, by spinning on the query.  That is no earlier
  // than the event itself, so completion times derived from it (and the
  // latencies) err on the late side, by the observation delay.
  e = hipEventCreate(&s->origin);
  if (e == hipSuccess) e = hipEventRecord(s->origin, s->stream);
  while (e == hipSuccess) {
    e = hipEventQuery(s->origin);
    if (e == hipErrorNotReady) e = hipSuccess;
    else break;
  }
  if (e != hipSuccess) return hip_fail(e, "clock origin");
  s->origin_ms = s->clock_ms();
  s->device_ready = true;
  return ADCT_OK;
}

const Tables* tables_for(adct_server* s, int kind, int n, int qstep) {
  const auto key = std::make_tuple(kind, n, qstep);
  auto it = s->tables.find(key);
  if (it != s->tables.end()) return &it->second;
  Tables t;
  if (build_tables_for(kind, n, qstep, &t) != ADCT_OK) return nullptr;
  return &s->tables.emplace(key, t).first->second;
}

template <int KIND, int DT>
void launch_class_typed(const ClassKey& c, dim3 grid, hipStream_t st, const SReq* r,
                        const int* b, int nq) {
  if (c.n == 8) {
    if (c.quant) serve8<KIND, DT, 64, true><<<grid, t8::kWave, 0, st>>>(r, b, nq);
    else if (c.rb == 10) serve8<KIND, DT, 10, false><<<grid, t8::kWave, 0, st>>>(r, b, nq);
    else if (c.rb == 28) serve8<KIND, DT, 28, false><<<grid, t8::kWave, 0, st>>>(r, b, nq);
    else serve8<KIND, DT, 64, false><<<grid, t8::kWave, 0, st>>>(r, b, nq);
  } else if (c.n == 16) {
    if (c.quant) serve_jam<KIND, 16, DT, true, 16><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
    else if (c.rb == 4) serve_jam<KIND, 16, DT, false, 4><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
    else if (c.rb == 8) serve_jam<KIND, 16, DT, false, 8><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
    else serve_jam<KIND, 16, DT, false, 16><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
  } else {
    if (c.quant) serve_jam<KIND, 32, DT, true, 32><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
    else if (c.rb == 4) serve_jam<KIND, 32, DT, false, 4><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
    else if (c.rb == 8) serve_jam<KIND, 32, DT, false, 8><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
    else serve_jam<KIND, 32, DT, false, 32><<<grid, jam::kBlock, 0, st>>>(r, b, nq);
  }
}

void launch_class(const ClassKey& c, int items, hipStream_t st, const SReq* r, const int* b,
                  int nq) {
  const dim3 grid(items);
  if (c.kind == KIND_SIGN) {
    if (c.dtype == ADCT_U8) launch_class_typed<KIND_SIGN, DT_U8>(c, grid, st, r, b, nq);
    else launch_class_typed<KIND_SIGN, DT_I16>(c, grid, st, r, b, nq);
  } else {
    if (c.dtype == ADCT_U8) launch_class_typed<KIND_ROUND, DT_U8>(c, grid, st, r, b, nq);
    else launch_class_typed<KIND_ROUND, DT_I16>(c, grid, st, r, b, nq);
  }
}

int do_submit(adct_server* s, const adct_request_t* req) {
  if (s == nullptr || req == nullptr) return set_error(ADCT_E_ARG, "server: null argument");
  if (int st = validate(*req)) return st;
  Member m;
  m.req = *req;
  layout(m);
  if (m.charge > s->budget) {
    ++s->n_refused;
    return set_error(ADCT_E_BUDGET, "server: request exceeds the whole budget");
  }
  if (s->charged + m.charge > s->budget || !s->ring_alloc(m.len, &m.off, &m.seq)) {
    ++s->n_refused;
    return set_error(ADCT_E_BUDGET, "server: budget full, retry after a poll");
  }
  s->charged += m.charge;
  s->queue.push_back(m);
  ++s->n_submitted;
  return set_error(ADCT_OK, "");
}

int do_flush(adct_server* s, int* launched) {
  if (launched) *launched = 0;
  if (s->queue.empty()) return set_error(ADCT_OK, "");
  if (int st = ensure_device(s)) return st;
  if (s->free_slots.empty()) return set_error(ADCT_OK, "");
  const int slot_id = s->free_slots.back();
  Slot& sl = s->slots[slot_id];
  const int m = static_cast<int>(std::min<size_t>(s->queue.size(), s->max_batch));
  sl.members.assign(s->queue.begin(), s->queue.begin() + m);

  // request table sorted by class; each class is one launch
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return class_of(sl.members[a].req) < class_of(sl.members[b].req);
  });
  struct Launch {
    ClassKey key;
    int first, count, items;
  };
  const TableLayout lay = table_layout(m);
  SReq* h_reqs = reinterpret_cast<SReq*>(sl.h_table);
  int* h_begins = reinterpret_cast<int*>(sl.h_table + lay.begins);
  memset(sl.h_table + lay.sse, 0, static_cast<size_t>(m) * sizeof(unsigned long long));
  SReq* d_reqs = reinterpret_cast<SReq*>(sl.d_table);
  const int* d_begins = reinterpret_cast<const int*>(sl.d_table + lay.begins);
  auto* d_sse = reinterpret_cast<unsigned long long*>(sl.d_table + lay.sse);
  std::vector<Launch> launches;
  for (int t = 0; t < m; ++t) {
    Member& mb = sl.members[order[t]];
    const adct_request_t& q = mb.req;
    const ClassKey key = class_of(q);
    if (launches.empty() || launches.back().key != key) launches.push_back({key, t, 0, 0});
    Launch& L = launches.back();
    const Tables* tb = tables_for(s, q.transform, q.n, q.qstep);
    if (tb == nullptr) return ADCT_E_ARG;
    const int tiles_x = q.width / q.n;
    const int tiles_y = q.height / q.n;
    const int gx = groups_x_of(q.n, tiles_x);
    SReq& rec = h_reqs[t];
    rec.src = q.d_src;
    rec.dst = s->arena + mb.off + mb.recon_off;
    rec.kept = reinterpret_cast<int32_t*>(s->arena + mb.off + mb.kept_off);
    rec.scaled = mb.scaled_off >= 0 ? reinterpret_cast<float*>(s->arena + mb.off + mb.scaled_off)
                                    : nullptr;
    rec.sse = d_sse + t;
    rec.pitch = q.pitch;
    rec.tiles_x = tiles_x;
    rec.groups_x = gx;
    rec.r = q.r;
    rec.pad = 0;
    rec.t = *tb;
    h_begins[t] = L.items;
    L.items += gx * tiles_y;
    ++L.count;
    mb.table = t;
  }
  // the slot's work follows whatever the caller's stream has queued (the inputs)
  const hipStream_t st = sl.stream;
  sl.launch_ms = s->clock_ms();
  hipError_t e = hipEventRecord(sl.ready, s->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, sl.ready, 0);
  // one upload: request records, first-item offsets and zeroed error energies
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.d_table, sl.h_table, lay.bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "request table upload");
  for (const Launch& L : launches)
    launch_class(L.key, L.items, st, d_reqs + L.first, d_begins + L.first, L.count);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "class launch");
  e = hipMemcpyAsync(sl.h_sse, d_sse, m * 8, hipMemcpyDeviceToHost, st);
  for (int i = 0; i < m && e == hipSuccess; ++i) {
    const Member& mb = sl.members[i];
    const adct_request_t& q = mb.req;
    const int esize = q.dtype == ADCT_U8 ? 1 : 2;
    if (q.h_kept != nullptr)
      e = hipMemcpyAsync(q.h_kept, s->arena + mb.off + mb.kept_off,
                         static_cast<int64_t>(q.height / q.n) * (q.width / q.n) * q.r * 4,
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && q.h_scaled != nullptr)
      e = hipMemcpyAsync(q.h_scaled, s->arena + mb.off + mb.scaled_off,
                         static_cast<int64_t>(q.height / q.n) * (q.width / q.n) * q.r * 4,
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && q.h_recon != nullptr)
      e = hipMemcpyAsync(q.h_recon, s->arena + mb.off + mb.recon_off,
                         static_cast<int64_t>(q.height) * q.pitch * esize, hipMemcpyDeviceToHost,
                         st);
  }
  if (e == hipSuccess) e = hipEventRecord(sl.done, st);
  if (e != hipSuccess) return hip_fail(e, "batch completion");
  s->queue.erase(s->queue.begin(), s->queue.begin() + m);
  s->free_slots.pop_back();
  sl.id = s->next_batch++;
  s->inflight.push_back(slot_id);
  s->max_seen = std::max<int64_t>(s->max_seen, m);
  if (launched) *launched = m;
  return set_error(ADCT_OK, "");
}

// Report the completed batches (in launch order among those complete) while
// their requests fit in out.
int do_poll(adct_server* s, int wait, adct_completion_t* out, int max_out, int* n_out) {
  if (n_out) *n_out = 0;
  for (const Member& mb : s->to_release) {
    s->ring_release(mb.seq);
    s->charged -= mb.charge;
  }
  s->to_release.clear();
  int n = 0;
  size_t i = 0;
  while (i < s->inflight.size()) {
    const int slot_id = s->inflight[i];
    Slot& sl = s->slots[slot_id];
    hipError_t e = wait ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (e != hipSuccess) return hip_fail(e, "batch completion");
    if (n + static_cast<int>(sl.members.size()) > max_out) break;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, s->origin, sl.done);
    if (e != hipSuccess) return hip_fail(e, "event time");
    const double done = s->origin_ms + ms;
    for (const Member& mb : sl.members) {
      adct_completion_t& c = out[n++];
      c.tag = mb.req.tag;
      c.batch = sl.id;
      c.sse = sl.h_sse[mb.table];
      c.done_ms = done;
      c.launch_ms = sl.launch_ms;
      c.d_kept = reinterpret_cast<const int32_t*>(s->arena + mb.off + mb.kept_off);
      c.d_scaled = mb.scaled_off >= 0
                       ? reinterpret_cast<const float*>(s->arena + mb.off + mb.scaled_off)
                       : nullptr;
      c.d_recon = s->arena + mb.off + mb.recon_off;
      s->to_release.push_back(mb);
    }
    s->n_completed += static_cast<int64_t>(sl.members.size());
    sl.members.clear();
    s->free_slots.push_back(slot_id);
    s->inflight.erase(s->inflight.begin() + i);
  }
  if (n_out) *n_out = n;
  return set_error(ADCT_OK, "");
}

}  // namespace

extern "C" {

ADCT_API int adct_server_create(int64_t budget_bytes, int max_inflight, int max_batch,
                                adct_stream_t stream, adct_server_t** server) {
  if (server == nullptr) return set_error(ADCT_E_ARG, "server: null output pointer");
  *server = nullptr;
  if (budget_bytes <= 0) return set_error(ADCT_E_ARG, "server: budget must be positive");
  if (max_inflight < 1 || max_inflight > 8)
    return set_error(ADCT_E_ARG, "server: max_inflight outside [1, 8]");
  if (max_batch < 1 || max_batch > kMaxBatch)
    return set_error(ADCT_E_ARG, "server: max_batch outside [1, 4096]");
  auto* s = new adct_server();
  s->budget = budget_bytes;
  s->max_inflight = max_inflight;
  s->max_batch = max_batch;
  s->stream = static_cast<hipStream_t>(stream);
  s->t0 = std::chrono::steady_clock::now();
  *server = s;
  return set_error(ADCT_OK, "");
}

ADCT_API int adct_server_destroy(adct_server_t* s) {
  if (s == nullptr) return set_error(ADCT_OK, "");
  int status = ADCT_OK;
  for (int id : s->inflight)
    if (hipEventSynchronize(s->slots[id].done) != hipSuccess) status = ADCT_E_HIP;
  for (Slot& sl : s->slots) {
    if (sl.d_table) (void)hipFree(sl.d_table);
    if (sl.h_table) (void)hipHostFree(sl.h_table);
    if (sl.h_sse) (void)hipHostFree(sl.h_sse);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.ready) (void)hipEventDestroy(sl.ready);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->origin) (void)hipEventDestroy(s->origin);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
  return status == ADCT_OK ? set_error(ADCT_OK, "")
                           : set_error(ADCT_E_HIP, "server: a batch failed while draining");
}

ADCT_API int adct_server_submit(adct_server_t* s, const adct_request_t* request) {
  return do_submit(s, request);
}

ADCT_API int adct_server_flush(adct_server_t* s, int* launched) {
  if (s == nullptr) return set_error(ADCT_E_ARG, "server: null server");
  return do_flush(s, launched);
}

ADCT_API int adct_server_poll(adct_server_t* s, int wait, adct_completion_t* out, int max_out,
                              int* n_out) {
  if (s == nullptr || out == nullptr || n_out == nullptr)
    return set_error(ADCT_E_ARG, "server: null argument");
  if (max_out < s->max_batch) return set_error(ADCT_E_ARG, "server: max_out below max_batch");
  return do_poll(s, wait, out, max_out, n_out);
}

ADCT_API int adct_server_stats(const adct_server_t* s, int64_t* out) {
  if (s == nullptr || out == nullptr) return set_error(ADCT_E_ARG, "server: null argument");
  int64_t in_flight = 0;
  for (int id : s->inflight) in_flight += static_cast<int64_t>(s->slots[id].members.size());
  out[0] = s->n_submitted;
  out[1] = s->n_completed;
  out[2] = s->next_batch;
  out[3] = static_cast<int64_t>(s->queue.size());
  out[4] = in_flight;
  out[5] = s->charged;
  out[6] = s->max_seen;
  out[7] = s->n_refused;
  return set_error(ADCT_OK, "");
}

ADCT_API double adct_server_clock_ms(const adct_server_t* s) {
  return s == nullptr ? 0.0 : s->clock_ms();
}

ADCT_API int adct_server_run_trace(adct_server_t* s, const adct_request_t* requests,
                                   const double* arrival_ms, int64_t n, double* latency_ms,
                                   int64_t* batch_of, uint64_t* sse, double* launch_ms) {
  if (s == nullptr || n < 0 || (n > 0 && (requests == nullptr || arrival_ms == nullptr)))
    return set_error(ADCT_E_ARG, "server: bad trace arguments");
  for (int64_t i = 1; i < n; ++i)
    if (arrival_ms[i] < arrival_ms[i - 1])
      return set_error(ADCT_E_ARG, "server: arrival times must be non-decreasing");
  if (!s->queue.empty() || !s->inflight.empty())
    return set_error(ADCT_E_ARG, "server: run_trace needs an idle server");
  if (n == 0) return set_error(ADCT_OK, "");
  if (int st = ensure_device(s)) return st;
  for (int64_t i = 0; i < n; ++i) {
    if (latency_ms) latency_ms[i] = NAN;
    if (launch_ms) launch_ms[i] = NAN;
    if (batch_of) batch_of[i] = -1;
    if (sse) sse[i] = 0;
  }
  std::vector<adct_completion_t> done(s->max_batch);
  std::deque<int64_t> waiting;
  int64_t next = 0, finished = 0;
  const double start = s->clock_ms();
  while (finished < n) {
    bool progress = false;
    int got = 0;
    if (int st = do_poll(s, 0, done.data(), s->max_batch, &got)) return st;
    for (int k = 0; k < got; ++k) {
      const int64_t i = done[k].tag;
      if (latency_ms) latency_ms[i] = done[k].done_ms - (start + arrival_ms[i]);
      if (launch_ms) launch_ms[i] = done[k].launch_ms - start;
      if (batch_of) batch_of[i] = done[k].batch;
      if (sse) sse[i] = done[k].sse;
    }
    finished += got;
    progress |= got > 0;
    const double now = s->clock_ms() - start;
    while (next < n && arrival_ms[next] <= now) waiting.push_back(next++);
    while (!waiting.empty()) {
      adct_request_t q = requests[waiting.front()];
      q.tag = waiting.front();
      const int st = do_submit(s, &q);
      if (st == ADCT_E_BUDGET) {
        Member probe;
        probe.req = q;
        layout(probe);
        if (probe.charge <= s->budget) break;   // wait for space
      }
      if (st != ADCT_OK) ++finished;           // invalid or never fits: NaN latency
      waiting.pop_front();
      progress = true;
    }
    int launched = 0;
    if (int st = do_flush(s, &launched)) return st;
    progress |= launched > 0;
    if (!progress) {
      if (s->inflight.empty() && s->queue.empty() && waiting.empty() && next < n) {
        const double gap = arrival_ms[next] - (s->clock_ms() - start);
        if (gap > 0.2)
          std::this_thread::sleep_for(std::chrono::microseconds(static_cast<int64_t>((gap - 0.1) * 1e3)));
      } else {
        std::this_thread::yield();
      }
    }
  }
  // release the last reported batch
  int got = 0;
  if (int st = do_poll(s, 1, done.data(), s->max_batch, &got)) return st;
  return set_error(ADCT_OK, "");
}

}  // extern "C"
