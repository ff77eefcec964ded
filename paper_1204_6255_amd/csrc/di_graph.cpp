// libdi host side: errors, device check, graph validation and upload.
//
// The graph input is the origin-sorted link list of Section 2.1. P is
// implied by it (Section 1): column j of P holds d/out_j at every link
// j -> i, out_j counting all links of j (self-loop included, Section 2.4).

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "di_internal.h"

namespace di {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

di_status check_device(int* device_out) {
  int count = 0;
  hipError_t err = hipGetDeviceCount(&count);
  if (err != hipSuccess || count <= 0) {
    set_error(std::string("no HIP device available (") +
              (err != hipSuccess ? hipGetErrorString(err) : "0 devices") +
              "); libdi has no CPU fallback");
    (void)hipGetLastError();
    return DI_E_DEVICE;
  }
  int dev = 0;
  DI_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  DI_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("libdi is built for gfx950, the current device is ") + prop.gcnArchName);
    return DI_E_DEVICE;
  }
  if (device_out) *device_out = dev;
  return DI_OK;
}

void free_workspace(Workspace* ws);

}  // namespace di

namespace {

void free_graph_device(di_graph* g) {
  void* ptrs[] = {g->row_ptr, g->col,    g->info,   g->csc_ptr,  g->csc_idx, g->row_lo,
                  g->it_r0,   g->it_r1,  g->it_l0,  g->it_l1,    g->it_seg,  g->heavy_row,
                  g->heavy_seg, g->hc_seg0, g->hc_seg1, g->hc_off, g->seg_heavy,
                  g->wp_col,  g->wp_info, g->hub_rank_node, g->hub_id_node, g->hub_id_rank};
  for (void* p : ptrs) (void)hipFree(p);
  for (int sh = 0; sh < di::kWinShapes; ++sh) {
    (void)hipFree(g->hub_tile[sh]);
    g->hub_tile[sh] = nullptr;
  }
  g->row_ptr = nullptr;
  g->col = nullptr;
  g->info = nullptr;
  g->csc_ptr = nullptr;
  g->csc_idx = nullptr;
  g->row_lo = nullptr;
  g->it_r0 = g->it_r1 = g->it_l0 = g->it_l1 = nullptr;
  g->it_seg = nullptr;
  g->heavy_row = nullptr;
  g->heavy_seg = nullptr;
  g->hc_seg0 = g->hc_seg1 = g->hc_off = nullptr;
  g->seg_heavy = nullptr;
  g->wp_col = nullptr;
  g->wp_info = nullptr;
  g->hub_rank_node = g->hub_id_node = g->hub_id_rank = nullptr;
}



template <typename V>
di_status upload(V** dst, const std::vector<V>& src) {
  const size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(V);
  hipError_t err = hipMalloc((void**)dst, bytes);
  if (err != hipSuccess) {
    *dst = nullptr;
    di::set_error(std::string("hipMalloc of ") + std::to_string(bytes) +
                  " bytes: " + hipGetErrorString(err));
    (void)hipGetLastError();
    return err == hipErrorOutOfMemory ? DI_E_NOMEM : DI_E_DEVICE;
  }
  if (!src.empty()) DI_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
  return DI_OK;
}

// Window-push layout (di_window.hip): each row's out-links with the near
// links (|i - j| <= kWinHalo) first and the far links after them, a far link
// into a ranked hub coded -1 - rank. Hubs are ranked by far in-links (at
// least kWinHubMinFar, ties to the lower id), at most kWinHubMax of them.
di_status build_window(di_graph* g, const std::vector<int64_t>& row_ptr,
                       const std::vector<int32_t>& col, const std::vector<uint32_t>& info) {
  const int64_t n = g->n;
  const int64_t W = di::kWinHalo;
  std::vector<int64_t> farin((size_t)n, 0);
  int64_t near_links = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int64_t j = col[e];
      if (j - i <= W && i - j <= W) ++near_links;
      else ++farin[j];
    }
  std::vector<int32_t> ranked;
  for (int64_t j = 0; j < n; ++j)
    if (farin[j] >= di::kWinHubMinFar) ranked.push_back((int32_t)j);
  auto by_far = [&](int32_t x, int32_t y) {
    return farin[x] != farin[y] ? farin[x] > farin[y] : x < y;
  };
  if ((int64_t)ranked.size() > di::kWinHubMax) {
    std::nth_element(ranked.begin(), ranked.begin() + di::kWinHubMax, ranked.end(), by_far);
    ranked.resize(di::kWinHubMax);
  }
  std::sort(ranked.begin(), ranked.end(), by_far);
  std::vector<int32_t> rank((size_t)n, -1);
  for (size_t r = 0; r < ranked.size(); ++r) rank[(size_t)ranked[r]] = (int32_t)r;
  std::vector<int32_t> wcol(col.size());
  std::vector<uint32_t> winfo((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t q = row_ptr[i];
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int64_t j = col[e];
      if (j - i <= W && i - j <= W) wcol[(size_t)q++] = (int32_t)j;
    }
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int64_t j = col[e];
      if (!(j - i <= W && i - j <= W))
        wcol[(size_t)q++] = rank[(size_t)j] >= 0 ? -1 - rank[(size_t)j] : (int32_t)j;
    }
    winfo[(size_t)i] = (info[(size_t)i] & (di::kOutMask | di::kLoopBit)) |
                       (rank[(size_t)i] >= 0 ? di::kHubBit : 0u);
  }
  std::vector<int32_t> id_node(ranked.begin(), ranked.end());
  std::sort(id_node.begin(), id_node.end());
  std::vector<int32_t> id_rank(id_node.size());
  for (size_t k = 0; k < id_node.size(); ++k) id_rank[k] = rank[(size_t)id_node[k]];
  g->n_hubs = (int64_t)ranked.size();
  g->near_links = near_links;
  di_status st = upload(&g->wp_col, wcol);
  if (st == DI_OK) st = upload(&g->wp_info, winfo);
  if (st == DI_OK) st = upload(&g->hub_rank_node, ranked);
  if (st == DI_OK) st = upload(&g->hub_id_node, id_node);
  if (st == DI_OK) st = upload(&g->hub_id_rank, id_rank);
  for (int sh = 0; sh < di::kWinShapes && st == DI_OK; ++sh) {
    const int64_t T = di::kWinTileOf[sh];
    const int64_t ntiles = (n + T - 1) / T;
    std::vector<int32_t> htile((size_t)ntiles + 1, 0);
    for (int32_t h : id_node) htile[(size_t)(h / T) + 1] += 1;
    for (int64_t t = 0; t < ntiles; ++t) htile[(size_t)t + 1] += htile[(size_t)t];
    // the window kernel keeps a tile's link offsets in 32 bits
    bool ok = true;
    for (int64_t t = 0; t < ntiles; ++t) {
      const int64_t a = t * T, b = std::min<int64_t>(a + T, n);
      if (row_ptr[(size_t)b] - row_ptr[(size_t)a] >= (int64_t(1) << 31)) ok = false;
    }
    g->n_wtiles[sh] = ntiles;
    g->window_ok[sh] = ok;
    st = upload(&g->hub_tile[sh], htile);
  }
  return st;
}

}  // namespace

extern "C" {

const char* di_last_error(void) { return di::g_error.c_str(); }

int32_t di_version(void) { return (1 << 16) | 0; }

void di_opts_default(di_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = DI_SOP;
  o->precision = DI_FP64;
  o->stop = DI_STOP_RESID;
  o->max_cycles = 100000;
  o->flags = 0;
  o->inner_tol = 1e-5;
  o->stream = nullptr;
}

di_status di_graph_create(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                          uint32_t flags, di_graph** out) {
  try {
    if (!out) {
      di::set_error("di_graph_create: out is NULL");
      return DI_E_INVAL;
    }
    *out = nullptr;
    if (n <= 0 || n > 0x7fffffffLL) {
      di::set_error("di_graph_create: n must be in [1, 2^31 - 1]");
      return DI_E_INVAL;
    }
    if (m < 0 || m >= (1LL << 33)) {
      di::set_error("di_graph_create: m must be in [0, 2^33)");
      return DI_E_INVAL;
    }
    if (m > 0 && (!src || !dst)) {
      di::set_error("di_graph_create: src or dst is NULL");
      return DI_E_INVAL;
    }
    if (flags != 0) {
      di::set_error("di_graph_create: flags must be 0");
      return DI_E_INVAL;
    }
    // validation, in one pass, before any device work
    for (int64_t e = 0; e < m; ++e) {
      const int64_t a = src[e], b = dst[e];
      if (a < 0 || a >= n || b < 0 || b >= n) {
        di::set_error("di_graph_create: link " + std::to_string(e) + " (" + std::to_string(a) +
                      " -> " + std::to_string(b) + ") has an id outside [0, n)");
        return DI_E_RANGE;
      }
      if (e > 0) {
        const int64_t pa = src[e - 1], pb = dst[e - 1];
        if (a < pa || (a == pa && b < pb)) {
          di::set_error("di_graph_create: links are not sorted by (origin, destination) at link " +
                        std::to_string(e));
          return DI_E_UNSORTED;
        }
        if (a == pa && b == pb) {
          di::set_error("di_graph_create: link " + std::to_string(a) + " -> " + std::to_string(b) +
                        " is listed twice");
          return DI_E_DUP;
        }
      }
    }
    int dev = 0;
    di_status st = di::check_device(&dev);
    if (st != DI_OK) return st;

    // host build: out-link lists without self-loops, per-node words, CSC
    std::vector<int64_t> row_ptr((size_t)n + 1, 0);
    std::vector<int64_t> outc((size_t)n, 0);
    std::vector<uint8_t> loopf((size_t)n, 0);
    int64_t n_loops = 0;
    for (int64_t e = 0; e < m; ++e) {
      const int32_t a = src[e];
      outc[a] += 1;
      if (a == dst[e]) {
        loopf[a] = 1;
        ++n_loops;
      } else {
        row_ptr[a + 1] += 1;
      }
    }
    std::vector<uint32_t> info((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
      if (outc[i] > (int64_t)di::kOutMask) {
        di::set_error("di_graph_create: node " + std::to_string(i) +
                      " has 2^30 or more out-links (not supported)");
        return DI_E_INVAL;
      }
      info[i] = (uint32_t)outc[i] | (loopf[i] ? di::kLoopBit : 0u);
    }
    std::vector<int64_t>().swap(outc);
    std::vector<uint8_t>().swap(loopf);
    int64_t n_dangling = 0, max_out = 0;
    for (int64_t i = 0; i < n; ++i) {
      row_ptr[i + 1] += row_ptr[i];
      const int64_t o = info[i] & di::kOutMask;
      n_dangling += o == 0;
      max_out = std::max(max_out, o);
    }
    const int64_t Lp = row_ptr[n];
    std::vector<int32_t> col((size_t)Lp);
    {
      int64_t q = 0;
      for (int64_t e = 0; e < m; ++e)
        if (src[e] != dst[e]) col[q++] = dst[e];
    }
    di_graph* g = new di_graph;
    g->n = n;
    g->L = m;
    g->Lp = Lp;
    g->n_dangling = n_dangling;
    g->n_loops = n_loops;
    g->max_out = max_out;
    g->device = dev;
    st = upload(&g->row_ptr, row_ptr);
    if (st == DI_OK) st = upload(&g->col, col);
    if (st == DI_OK) st = upload(&g->info, info);
    if (st == DI_OK) st = build_window(g, row_ptr, col, info);
    std::vector<int64_t>().swap(row_ptr);
    std::vector<int32_t>().swap(col);
    if (st == DI_OK) {
      // in-links without self-loops (rows of P), ascending origin per row
      std::vector<int64_t> cptr((size_t)n + 1, 0);
      for (int64_t e = 0; e < m; ++e)
        if (src[e] != dst[e]) cptr[dst[e] + 1] += 1;
      int64_t max_in = 0;
      for (int64_t i = 0; i < n; ++i) {
        max_in = std::max(max_in, cptr[i + 1]);
        cptr[i + 1] += cptr[i];
      }
      g->max_in = max_in;
      std::vector<int32_t> cidx((size_t)Lp);
      {
        std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t e = 0; e < m; ++e)
          if (src[e] != dst[e]) cidx[fill[dst[e]]++] = src[e];
      }
      // pull work items: runs of whole rows with at most kPullChunk in-links
      // and kPullMaxRows rows; a row with more in-links is split into
      // segments of kPullChunk links, summed separately
      std::vector<int64_t> r0v, r1v, l0v, l1v, hseg;
      std::vector<int32_t> segv, hrow, seg_heavy;
      int64_t nseg = 0, open_r0 = -1, cur_links = 0, cur_rows = 0;
      std::vector<uint16_t> rlo((size_t)n, 0);
      auto flush = [&](int64_t end_row) {
        if (open_r0 < 0) return;
        for (int64_t r = open_r0; r < end_row; ++r)
          rlo[(size_t)r] = (uint16_t)(cptr[r] - cptr[open_r0]);
        r0v.push_back(open_r0);
        r1v.push_back(end_row);
        l0v.push_back(cptr[open_r0]);
        l1v.push_back(cptr[end_row]);
        segv.push_back(-1);
        open_r0 = -1;
        cur_links = cur_rows = 0;
      };
      for (int64_t j = 0; j < n; ++j) {
        const int64_t deg = cptr[j + 1] - cptr[j];
        if (deg > di::kPullChunk) {
          flush(j);
          hrow.push_back((int32_t)j);
          hseg.push_back(nseg);
          info[j] |= di::kHeavyBit;
          for (int64_t lo = cptr[j]; lo < cptr[j + 1]; lo += di::kPullChunk) {
            r0v.push_back(j);
            r1v.push_back(j + 1);
            l0v.push_back(lo);
            l1v.push_back(std::min<int64_t>(lo + di::kPullChunk, cptr[j + 1]));
            segv.push_back((int32_t)nseg++);
            seg_heavy.push_back((int32_t)(hrow.size() - 1));
          }
          continue;
        }
        if (open_r0 >= 0 && (cur_links + deg > di::kPullChunk || cur_rows >= di::kPullMaxRows))
          flush(j);
        if (open_r0 < 0) open_r0 = j;
        cur_links += deg;
        cur_rows += 1;
      }
      flush(n);
      hseg.push_back(nseg);
      g->n_items = (int64_t)r0v.size();
      g->n_heavy = (int64_t)hrow.size();
      g->n_segs = nseg;
      // completion chunks of at most kHeavyChunkSegs segment sums
      std::vector<int32_t> hc0, hc1, hoff;
      for (size_t h = 0; h < hrow.size(); ++h) {
        hoff.push_back((int32_t)hc0.size());
        for (int64_t q = hseg[h]; q < hseg[h + 1]; q += di::kHeavyChunkSegs) {
          hc0.push_back((int32_t)q);
          hc1.push_back((int32_t)std::min<int64_t>(q + di::kHeavyChunkSegs, hseg[h + 1]));
        }
      }
      hoff.push_back((int32_t)hc0.size());
      g->n_hchunks = (int64_t)hc0.size();
      g->heavy_atomic = g->n_heavy > di::kHeavyLds || g->n_hchunks > di::kHeavyLds;
      st = upload(&g->csc_ptr, cptr);
      if (st == DI_OK) st = upload(&g->csc_idx, cidx);
      if (st == DI_OK) st = upload(&g->row_lo, rlo);
      if (st == DI_OK) st = upload(&g->it_r0, r0v);
      if (st == DI_OK) st = upload(&g->it_r1, r1v);
      if (st == DI_OK) st = upload(&g->it_l0, l0v);
      if (st == DI_OK) st = upload(&g->it_l1, l1v);
      if (st == DI_OK) st = upload(&g->it_seg, segv);
      if (st == DI_OK) st = upload(&g->heavy_row, hrow);
      if (st == DI_OK) st = upload(&g->heavy_seg, hseg);
      if (st == DI_OK) st = upload(&g->hc_seg0, hc0);
      if (st == DI_OK) st = upload(&g->hc_seg1, hc1);
      if (st == DI_OK) st = upload(&g->hc_off, hoff);
      if (st == DI_OK) st = upload(&g->seg_heavy, seg_heavy);
      // the node words carry the heavy flags
      if (st == DI_OK)
        DI_HIP(hipMemcpy(g->info, info.data(), info.size() * sizeof(uint32_t), hipMemcpyHostToDevice));

    }
    if (st != DI_OK) {
      free_graph_device(g);
      delete g;
      return st;
    }
    *out = g;
    return DI_OK;
  } catch (const std::bad_alloc&) {
    di::set_error("di_graph_create: host allocation failed");
    return DI_E_NOMEM;
  } catch (...) {
    di::set_error("di_graph_create: unexpected exception");
    return DI_E_INVAL;
  }
}

void di_graph_destroy(di_graph* g) {
  if (!g) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != g->device) (void)hipSetDevice(g->device);
  {
    std::lock_guard<std::mutex> lock(g->mu);
    for (di::Workspace* ws : g->pool) di::free_workspace(ws);
    g->pool.clear();
    for (di::BatchWs* ws : g->bpool) di::free_batch_ws(ws);
    g->bpool.clear();
  }
  free_graph_device(g);
  if (cur != g->device) (void)hipSetDevice(cur);
  delete g;
}

di_status di_graph_info(const di_graph* g, int64_t* n, int64_t* m, int64_t* n_dangling,
                        int64_t* n_loops) {
  if (!g) {
    di::set_error("di_graph_info: graph is NULL");
    return DI_E_INVAL;
  }
  if (n) *n = g->n;
  if (m) *m = g->L;
  if (n_dangling) *n_dangling = g->n_dangling;
  if (n_loops) *n_loops = g->n_loops;
  return DI_OK;
}

}  // extern "C"
