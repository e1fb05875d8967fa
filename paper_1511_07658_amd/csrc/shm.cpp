#include "shm.hpp"

#include <errno.h>
#include <fcntl.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstring>

#include "common.hpp"

namespace gvm {

std::string ctl_object_name(const std::string& ns) { return "/" + ns + ".ctl"; }
std::string data_object_name(const std::string& ns, int rank) { return "/" + ns + ".r" + std::to_string(rank); }
std::string default_namespace() { return "gvm." + std::to_string(static_cast<unsigned>(getuid())); }

int Segment::create(const std::string& nm, uint64_t sz) {
  close();
  shm_unlink(nm.c_str());  // a stale object of a dead manager
  int fd = shm_open(nm.c_str(), O_CREAT | O_EXCL | O_RDWR, 0600);
  if (fd < 0) return fail(GVM_ESYS, "shm_open(%s): %s", nm.c_str(), strerror(errno));
  if (ftruncate(fd, static_cast<off_t>(sz)) != 0) {
    int e = errno;
    ::close(fd);
    shm_unlink(nm.c_str());
    return fail(GVM_ESYS, "ftruncate(%s, %llu): %s", nm.c_str(), (unsigned long long)sz, strerror(e));
  }
  void* p = mmap(nullptr, sz, PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
  ::close(fd);
  if (p == MAP_FAILED) {
    int e = errno;
    shm_unlink(nm.c_str());
    return fail(GVM_ESYS, "mmap(%s): %s", nm.c_str(), strerror(e));
  }
  addr = p;
  bytes = sz;
  name = nm;
  owner = true;
  return GVM_OK;
}

int Segment::open(const std::string& nm) {
  close();
  int fd = shm_open(nm.c_str(), O_RDWR, 0600);
  if (fd < 0) return fail(GVM_ESYS, "shm_open(%s): %s", nm.c_str(), strerror(errno));
  struct stat st;
  if (fstat(fd, &st) != 0) {
    int e = errno;
    ::close(fd);
    return fail(GVM_ESYS, "fstat(%s): %s", nm.c_str(), strerror(e));
  }
  void* p = mmap(nullptr, static_cast<size_t>(st.st_size), PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
  ::close(fd);
  if (p == MAP_FAILED) return fail(GVM_ESYS, "mmap(%s): %s", nm.c_str(), strerror(errno));
  addr = p;
  bytes = static_cast<uint64_t>(st.st_size);
  name = nm;
  owner = false;
  return GVM_OK;
}

void Segment::close() {
  if (addr) munmap(addr, bytes);
  if (owner && !name.empty()) shm_unlink(name.c_str());
  addr = nullptr;
  bytes = 0;
  owner = false;
  name.clear();
}

}  // namespace gvm
