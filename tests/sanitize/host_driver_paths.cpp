// Sanitizer harness (ASan + UBSan on host code) for the library's host-only
// paths: argument checks, the measuring pass that lays out the arena of
// dashsvd_run and dashsvd_run_batched (dashsvd_workspace_size*), status
// strings and the failure path of dashsvd_create without a device.  No GPU
// is touched.  Built and run by tests/test_sanitize_host.py.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "dashsvd.h"

namespace {

struct HostCsr {
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<float> val;
  dashsvd_csr c{};
};

// rows r of an m x n matrix with (r % 5) + 1 nonzeros at columns r, r+1, ...
HostCsr make(int64_t m, int64_t n) {
  HostCsr h;
  h.rp.push_back(0);
  for (int64_t r = 0; r < m; ++r) {
    const int64_t d = (r % 5) + 1 < n ? (r % 5) + 1 : n;
    for (int64_t j = 0; j < d; ++j) {
      h.col.push_back((int32_t)((r + j) % n));
      h.val.push_back(1.0f + (float)j);
    }
    // columns strictly increasing inside the row
    std::sort(h.col.end() - d, h.col.end());
    h.rp.push_back((int64_t)h.col.size());
  }
  h.c.m = m;
  h.c.n = n;
  h.c.nnz = (int64_t)h.col.size();
  h.c.row_ptr = h.rp.data();
  h.c.col_idx = h.col.data();
  h.c.values = h.val.data();
  h.c.value_dtype = DASHSVD_F32;
  h.c.on_device = 0;
  return h;
}

int expect(bool ok, const char *what) {
  if (!ok) std::printf("FAILED: %s\n", what);
  return ok ? 0 : 1;
}

}  // namespace

int main() {
  int bad = 0;
  size_t bytes = 0;
  // the measuring pass of single solves: tall, wide, every precision
  const int64_t shapes[][2] = {{5000, 3000}, {700, 2100}, {64, 64}, {1, 300}};
  for (auto &s : shapes) {
    HostCsr A = make(s[0], s[1]);
    for (int prec = 0; prec <= 2; ++prec) {
      const int k = s[0] < 20 ? 0 : 8;
      const dashsvd_status st = dashsvd_workspace_size(&A.c, k > 0 ? k : 1, 4, prec, &bytes);
      const bool fits = (k > 0 ? k : 1) + 4 <= (s[0] < s[1] ? s[0] : s[1]);
      bad |= expect(fits ? (st == DASHSVD_OK && bytes > 0) : st == DASHSVD_ERR_INVALID_ARG, "workspace_size");
    }
  }
  // the batched layout: uneven members, tall and square
  std::vector<HostCsr> mats;
  for (int i = 0; i < 37; ++i) mats.push_back(make(200 + 37 * i, 150 + 11 * i));
  std::vector<dashsvd_csr> arr;
  for (auto &m : mats) arr.push_back(m.c);
  for (int prec = 0; prec <= 2; ++prec)
    bad |= expect(dashsvd_workspace_size_batched(arr.data(), (int32_t)arr.size(), 8, 4, prec, &bytes) == DASHSVD_OK &&
                      bytes > 0,
                  "workspace_size_batched");
  // argument errors
  HostCsr A = make(100, 80);
  bad |= expect(dashsvd_workspace_size(&A.c, 0, 4, 0, &bytes) == DASHSVD_ERR_INVALID_ARG, "k = 0");
  bad |= expect(dashsvd_workspace_size(&A.c, 8, 0, 0, &bytes) == DASHSVD_ERR_INVALID_ARG, "s = 0");
  bad |= expect(dashsvd_workspace_size(&A.c, 70, 20, 0, &bytes) == DASHSVD_ERR_INVALID_ARG, "l > min(m, n)");
  bad |= expect(dashsvd_workspace_size(nullptr, 8, 4, 0, &bytes) == DASHSVD_ERR_INVALID_ARG, "null matrix");
  bad |= expect(dashsvd_workspace_size(&A.c, 8, 4, 7, &bytes) == DASHSVD_ERR_INVALID_ARG, "precision");
  for (int s = -7; s <= 3; ++s) bad |= expect(dashsvd_status_string((dashsvd_status)s) != nullptr, "status string");
  // no device here: create fails cleanly and says why
  dashsvd_handle *h = nullptr;
  const dashsvd_status st = dashsvd_create(&h, nullptr);
  if (st == DASHSVD_OK) {
    dashsvd_destroy(h);
  } else {
    bad |= expect(h == nullptr && dashsvd_last_error(nullptr)[0] != 0, "create without a device");
  }
  std::printf("host driver paths: %s\n", bad ? "FAILED" : "ok");
  return bad;
}
