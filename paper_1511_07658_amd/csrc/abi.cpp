// extern "C" entry points of libgvm.so (declared in include/gvm.h).
#include <cstring>
#include <mutex>
#include <string>

#include "common.hpp"
#include "gvm.h"
#include "manager.hpp"
#include "rank.hpp"

namespace {
std::mutex g_mgr_mu;
gvm::Manager* g_mgr = nullptr;
}  // namespace

extern "C" {

void gvm_config_default(gvm_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->size = sizeof(gvm_config);
  cfg->nranks = 8;
  cfg->shm_bytes_per_rank = 64ull << 20;
  cfg->hbm_budget_bytes = 16ull << 30;
  cfg->staging_bytes = 0;
  cfg->mode = GVM_MODE_BATCH;
  cfg->policy = GVM_POLICY_AUTO;
  cfg->batch_window_us = 2000;
  cfg->max_inflight = 0;
  cfg->nstreams = 0;
  cfg->use_graphs = 0;
  cfg->backend = GVM_BACKEND_HIP;
  cfg->copy_threads = 4;
  cfg->bs_rate = 0.02f;
  cfg->bs_volatility = 0.30f;
  cfg->small_request_bytes = 8u << 20;
  cfg->early_copy_in = 1;
  cfg->name[0] = 0;
}

int gvm_cu_partition_masks(uint32_t latency_cus, uint32_t* latency_mask, uint32_t* bulk_mask) {
  gvm::clear_error();
  if (!latency_mask || !bulk_mask) return gvm::fail(GVM_EINVAL, "mask pointer is NULL");
  const int rc = gvm::cu_partition_masks(latency_cus, latency_mask, bulk_mask);
  if (rc != GVM_OK) return gvm::fail(rc, "latency_cus must be a multiple of 32 in 32..224");
  return GVM_OK;
}

int gvm_init(const gvm_config* cfg) {
  gvm::clear_error();
  if (!cfg) return gvm::fail(GVM_EINVAL, "cfg is NULL");
  std::lock_guard<std::mutex> lk(g_mgr_mu);
  if (g_mgr) return gvm::fail(GVM_ESTATE, "a manager already runs in this process");
  auto* m = new gvm::Manager();
  int rc = m->init(*cfg);
  if (rc != GVM_OK) {
    delete m;
    return rc;
  }
  g_mgr = m;
  return GVM_OK;
}

int gvm_attach(int rank) {
  gvm::clear_error();
  return gvm::rank_attach(nullptr, rank);
}

int gvm_attach_ns(const char* name, int rank) {
  gvm::clear_error();
  return gvm::rank_attach(name, rank);
}

int64_t gvm_submit(int rank, int kernel_id, const void* in, void* out, uint64_t n) {
  gvm::clear_error();
  return gvm::rank_submit(rank, kernel_id, in, out, n, 0);
}

int64_t gvm_submit_ex(int rank, int kernel_id, const void* in, void* out, uint64_t n, uint32_t flags) {
  gvm::clear_error();
  return gvm::rank_submit(rank, kernel_id, in, out, n, flags);
}

int gvm_wait(int rank, int64_t ticket, int64_t timeout_ns) {
  gvm::clear_error();
  return gvm::rank_wait(rank, ticket, timeout_ns);
}

int gvm_wait_timed(int rank, int64_t ticket, int64_t timeout_ns, uint64_t* ts) {
  gvm::clear_error();
  if (ticket < 0) return gvm::fail(GVM_EINVAL, "gvm_wait_timed needs one ticket");
  return gvm::rank_wait(rank, ticket, timeout_ns, ts);
}

int gvm_wait_any(int rank, int64_t timeout_ns, int64_t* ticket_out) {
  gvm::clear_error();
  return gvm::rank_wait_any(rank, timeout_ns, ticket_out);
}

int gvm_wait_any_timed(int rank, int64_t timeout_ns, int64_t* ticket_out, uint64_t* ts) {
  gvm::clear_error();
  return gvm::rank_wait_any(rank, timeout_ns, ticket_out, ts);
}

int gvm_detach(int rank) {
  gvm::clear_error();
  return gvm::rank_detach(rank);
}

int gvm_shutdown(void) {
  gvm::clear_error();
  int rc = gvm::rank_detach_all();
  std::lock_guard<std::mutex> lk(g_mgr_mu);
  if (g_mgr) {
    int rc2 = g_mgr->shutdown();
    delete g_mgr;
    g_mgr = nullptr;
    if (rc == GVM_OK) rc = rc2;
  }
  return rc;
}

void* gvm_rank_buffer(int rank, uint64_t bytes) {
  gvm::clear_error();
  return gvm::rank_buffer(rank, bytes);
}

int gvm_stats_json(char* buf, uint64_t cap) {
  gvm::clear_error();
  std::lock_guard<std::mutex> lk(g_mgr_mu);
  if (!g_mgr) return gvm::fail(GVM_ESTATE, "no manager runs in this process");
  std::string s;
  int rc = g_mgr->stats_json(&s);
  if (rc != GVM_OK) return rc;
  if (buf && cap > 0) {
    const size_t n = s.size() < cap - 1 ? s.size() : static_cast<size_t>(cap - 1);
    memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return static_cast<int>(s.size());
}

int gvm_stats_reset(void) {
  gvm::clear_error();
  std::lock_guard<std::mutex> lk(g_mgr_mu);
  if (!g_mgr) return gvm::fail(GVM_ESTATE, "no manager runs in this process");
  g_mgr->reset_stats();
  return GVM_OK;
}

int gvm_trace_dump(const char* path) {
  gvm::clear_error();
  std::lock_guard<std::mutex> lk(g_mgr_mu);
  if (!g_mgr) return gvm::fail(GVM_ESTATE, "no manager runs in this process");
  return g_mgr->trace_dump(path);
}

const char* gvm_last_error(void) { return gvm::last_error_text(); }

}  // extern "C"
