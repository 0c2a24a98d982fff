// Host side of a sparse X: validation of the compressed rows, the transposed
// copy (compressed columns, rows ascending within each column, so the X^T A
// product sums in a fixed order) and the work partition of the products of
// k_sparse.hip, uploaded once per matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "enmf_internal.h"

using namespace enmf;

const SparseX* enmf::sparse_of(const enmf_matrix* X) {
  if (X->dtype != ENMF_CSR) return nullptr;
  return static_cast<const SparseX*>(reinterpret_cast<const enmf_sparse*>(X->data));
}

namespace {

struct HostForm {
  int64_t rows = 0, cols = 0, nnz = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<float> val;
  std::vector<int64_t> item_p0, item_p1;
  std::vector<int32_t> item_row, item_slot, split_row, split_s0;
  int64_t nslots = 0;
};

// Work items: the stored entries of a row, cut where the column crosses into
// the next panel of `panel` columns (0: no panels) and after kSpChunk
// entries; an empty row is one empty item.  A row of one item writes its
// output row directly, the items of a longer row take consecutive slots.
// The items are then ordered by panel (rows ascending within a panel), so the
// blocks running at any moment gather from one panel's rows of the factor
// (kSpPanel rows of 40 floats, 10 MB, stay in the last-level cache).
void partition(HostForm& h, int64_t panel) {
  struct Piece {
    int64_t pan, p0, p1;
    int32_t row, slot;
  };
  std::vector<Piece> pcs, cur;
  pcs.reserve((size_t)h.rows + (size_t)(h.nnz / 8));
  int32_t slot = 0;
  for (int64_t i = 0; i < h.rows; ++i) {
    const int64_t a = h.ptr[i], b = h.ptr[i + 1];
    cur.clear();
    if (a == b) cur.push_back({0, a, a, (int32_t)i, -1});
    for (int64_t p = a; p < b;) {
      const int64_t pan = panel > 0 ? h.idx[p] / panel : 0;
      const int64_t lim = b - p < kSpChunk ? b : p + kSpChunk;
      int64_t q = p + 1;
      while (q < lim && (panel == 0 || h.idx[q] / panel == pan)) ++q;
      cur.push_back({pan, p, q, (int32_t)i, -1});
      p = q;
    }
    if (cur.size() > 1) {
      h.split_row.push_back((int32_t)i);
      h.split_s0.push_back(slot);
      for (Piece& c : cur) c.slot = slot++;
    }
    pcs.insert(pcs.end(), cur.begin(), cur.end());
  }
  h.split_s0.push_back(slot);
  h.nslots = slot;
  std::stable_sort(pcs.begin(), pcs.end(),
                   [](const Piece& x, const Piece& y) { return x.pan < y.pan; });
  for (const Piece& c : pcs) {
    h.item_p0.push_back(c.p0);
    h.item_p1.push_back(c.p1);
    h.item_row.push_back(c.row);
    h.item_slot.push_back(c.slot);
  }
}

// Compressed columns of the CSR matrix `a`, rows ascending within a column.
void transpose(const HostForm& a, HostForm& t) {
  t.rows = a.cols;
  t.cols = a.rows;
  t.nnz = a.nnz;
  t.ptr.assign(t.rows + 1, 0);
  for (int64_t p = 0; p < a.nnz; ++p) t.ptr[a.idx[p] + 1] += 1;
  for (int64_t j = 0; j < t.rows; ++j) t.ptr[j + 1] += t.ptr[j];
  std::vector<int64_t> next(t.ptr.begin(), t.ptr.end() - 1);
  t.idx.resize(a.nnz);
  t.val.resize(a.nnz);
  for (int64_t i = 0; i < a.rows; ++i) {
    for (int64_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      const int64_t q = next[a.idx[p]]++;
      t.idx[q] = (int32_t)i;
      t.val[q] = a.val[p];
    }
  }
}

void free_form(SparseForm& f) {
  void* ps[] = {f.ptr,      f.idx,       f.val,       f.item_p0, f.item_p1,
                f.item_row, f.item_slot, f.split_row, f.split_s0};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  f = SparseForm();
}

template <typename T>
bool upload(T** dst, const std::vector<T>& src, hipStream_t s) {
  const size_t bytes = src.size() * sizeof(T);
  if (hipMalloc(reinterpret_cast<void**>(dst), bytes < 256 ? 256 : bytes) != hipSuccess) {
    (void)hipGetLastError();
    *dst = nullptr;
    return false;
  }
  if (bytes == 0) return true;
  return hipMemcpyAsync(*dst, src.data(), bytes, hipMemcpyHostToDevice, s) == hipSuccess;
}

bool upload_form(const HostForm& h, SparseForm& f, hipStream_t s) {
  f.rows = h.rows;
  f.cols = h.cols;
  f.nnz = h.nnz;
  f.nitems = (int64_t)h.item_row.size();
  f.nslots = h.nslots;
  f.nsplit = (int64_t)h.split_row.size();
  return upload(&f.ptr, h.ptr, s) && upload(&f.idx, h.idx, s) && upload(&f.val, h.val, s) &&
         upload(&f.item_p0, h.item_p0, s) && upload(&f.item_p1, h.item_p1, s) &&
         upload(&f.item_row, h.item_row, s) &&
         upload(&f.item_slot, h.item_slot, s) && upload(&f.split_row, h.split_row, s) &&
         upload(&f.split_s0, h.split_s0, s);
}

enmf_status bad(enmf_ctx* c, const std::string& msg) {
  ctx_set_error(c, msg.c_str());
  return ENMF_EINVAL;
}

}  // namespace

extern "C" {

enmf_status enmf_sparse_create(enmf_ctx* c, int64_t m, int64_t n, int64_t nnz,
                               const int64_t* rowptr, const int32_t* colind, const float* vals,
                               enmf_sparse** out) {
  if (!c || !out) return ENMF_EINVAL;
  *out = nullptr;
  ctx_set_error(c, "");
  if (hipSetDevice(ctx_device(c)) != hipSuccess) {
    ctx_set_error(c, "hipSetDevice failed");
    return ENMF_EDEVICE;
  }
  if (!rowptr || (nnz > 0 && (!colind || !vals))) return bad(c, "null pointer");
  if (m < 1 || n < 1 || m > INT32_MAX || n > INT32_MAX || nnz < 0)
    return bad(c, "sparse X needs 1 <= m, n < 2^31 and nnz >= 0");
  if (rowptr[0] != 0 || rowptr[m] != nnz) return bad(c, "rowptr must run from 0 to nnz");
  for (int64_t i = 0; i < m; ++i) {
    const int64_t a = rowptr[i], b = rowptr[i + 1];
    if (b < a || b > nnz) return bad(c, "rowptr decreases or exceeds nnz at row " + std::to_string(i));
    for (int64_t p = a; p < b; ++p) {
      if (colind[p] < 0 || colind[p] >= n)
        return bad(c, "column index out of range in row " + std::to_string(i));
      if (p > a && colind[p] <= colind[p - 1])
        return bad(c, "column indices must increase strictly within row " + std::to_string(i));
      if (!std::isfinite(vals[p])) return bad(c, "non-finite value in row " + std::to_string(i));
    }
  }
  HostForm a, t;
  a.rows = m;
  a.cols = n;
  a.nnz = nnz;
  a.ptr.assign(rowptr, rowptr + m + 1);
  a.idx.assign(colind, colind + nnz);
  a.val.assign(vals, vals + nnz);
  transpose(a, t);
  partition(a, kSpPanel);
  partition(t, kSpPanel);
  hipStream_t s = ctx_stream(c);
  enmf_sparse* sp = new enmf_sparse();
  sp->device = ctx_device(c);
  const bool ok = upload_form(a, sp->csr, s) && upload_form(t, sp->csc, s);
  const bool synced = hipStreamSynchronize(s) == hipSuccess;
  if (!ok || !synced) {
    (void)hipGetLastError();
    free_form(sp->csr);
    free_form(sp->csc);
    delete sp;
    ctx_set_error(c, "device copies of the sparse X could not be allocated or written");
    return ENMF_ENOMEM;
  }
  *out = sp;
  return ENMF_OK;
}

void enmf_sparse_destroy(enmf_sparse* sp) {
  if (!sp || sp->magic != kSparseMagic) return;
  (void)hipSetDevice(sp->device);
  free_form(sp->csr);
  free_form(sp->csc);
  sp->magic = 0;
  delete sp;
}

}  // extern "C"
