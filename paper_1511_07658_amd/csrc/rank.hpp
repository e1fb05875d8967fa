// Rank side of the C-ABI (implemented in rank.cpp).
#pragma once

#include <cstdint>

namespace gvm {

int rank_attach(const char* name, int rank);
int64_t rank_submit(int rank, int kernel_id, const void* in, void* out, uint64_t n, uint32_t flags);
int rank_wait(int rank, int64_t ticket, int64_t timeout_ns, uint64_t* ts = nullptr);
int rank_wait_any(int rank, int64_t timeout_ns, int64_t* ticket_out, uint64_t* ts = nullptr);
int rank_detach(int rank);
int rank_detach_all();
void* rank_buffer(int rank, uint64_t bytes);

}  // namespace gvm
