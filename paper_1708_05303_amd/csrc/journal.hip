// Batch journal: one checksummed record per finished mock, so that a batch of
// mock catalogues (the covariance runs that the modal compression of Sec. 3.5
// makes cheap) can be stopped at any point and resumed without recomputing
// the mocks already done. Host code only.
//
// File layout (little endian):
//   header  16 bytes: "BSPJRNL" NUL, u32 format version, u32 zero
//   record  48-byte head: u32 magic, u32 has_beta, u64 key, u64 config hash,
//           i64 particle count, i32 nl, i32 ntri, i32 d, i32 zero
//           payload: f64 B[nl*ntri], f64 alpha[d], f64 beta[d] if has_beta
//           u64 FNV-1a 64 of the head and the payload
// A record is written with one write call at the end of the valid prefix; a
// process killed during that call leaves a torn record, which the next open
// finds by its length or checksum and cuts off.
#include <fcntl.h>
#include <sys/file.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstring>
#include <string>
#include <vector>

#include "bsp_internal.h"

namespace bsp {

namespace {

constexpr char kMagic[8] = {'B', 'S', 'P', 'J', 'R', 'N', 'L', 0};
constexpr uint32_t kVersion = 1;
constexpr uint32_t kRecMagic = 0x43455242u;  // "BREC"
constexpr size_t kHead = 48, kFileHead = 16;

struct RecHead {
  uint32_t magic, has_beta;
  uint64_t key, hash;
  int64_t np;
  int32_t nl, ntri, d, zero;
};
static_assert(sizeof(RecHead) == kHead, "record head layout");

bool read_at(int fd, void* buf, size_t n, int64_t off) {
  char* p = static_cast<char*>(buf);
  while (n) {
    const ssize_t r = ::pread(fd, p, n, off);
    if (r < 0 && errno == EINTR) continue;
    if (r <= 0) return false;
    p += r;
    n -= (size_t)r;
    off += r;
  }
  return true;
}

bool write_at(int fd, const void* buf, size_t n, int64_t off) {
  const char* p = static_cast<const char*>(buf);
  while (n) {
    const ssize_t r = ::pwrite(fd, p, n, off);
    if (r < 0 && errno == EINTR) continue;
    if (r <= 0) return false;
    p += r;
    n -= (size_t)r;
    off += r;
  }
  return true;
}

std::string sys_err(const std::string& what, const std::string& path) {
  return what + " " + path + ": " + std::strerror(errno);
}

}  // namespace

uint64_t fnv1a64(const void* data, size_t n, uint64_t h) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

int64_t journal_payload_doubles(int nl, int ntri, int d, int has_beta) {
  return (int64_t)nl * ntri + (int64_t)d * (has_beta ? 2 : 1);
}

Journal::~Journal() { close(); }

void Journal::close() {
  if (fd_ >= 0) {
    ::flock(fd_, LOCK_UN);
    ::close(fd_);
  }
  fd_ = -1;
  recs_.clear();
  valid_bytes_ = file_bytes_ = 0;
}

bool Journal::open(const std::string& path, bool create, std::string& err) {
  close();
  path_ = path;
  fd_ = ::open(path.c_str(), create ? (O_RDWR | O_CREAT) : O_RDONLY, 0644);
  if (fd_ < 0) {
    err = sys_err("cannot open journal", path);
    return false;
  }
  // one writer at a time: a second batch on the same journal would interleave records
  if (::flock(fd_, (create ? LOCK_EX : LOCK_SH) | LOCK_NB) != 0) {
    err = sys_err("journal is locked by another process", path);
    ::close(fd_);
    fd_ = -1;
    return false;
  }
  struct stat st;
  if (::fstat(fd_, &st) != 0) {
    err = sys_err("cannot stat journal", path);
    close();
    return false;
  }
  file_bytes_ = st.st_size;
  if (file_bytes_ == 0) {
    if (create) {
      unsigned char h[kFileHead] = {};
      std::memcpy(h, kMagic, 8);
      std::memcpy(h + 8, &kVersion, 4);
      if (!write_at(fd_, h, kFileHead, 0)) {
        err = sys_err("cannot write journal header", path);
        close();
        return false;
      }
      file_bytes_ = kFileHead;
    }
    valid_bytes_ = file_bytes_;
    return true;
  }
  unsigned char h[kFileHead];
  uint32_t ver = 0;
  if (file_bytes_ < (int64_t)kFileHead || !read_at(fd_, h, kFileHead, 0) || std::memcmp(h, kMagic, 8) != 0 ||
      (std::memcpy(&ver, h + 8, 4), ver != kVersion)) {
    err = "not a batch journal (or another format version): " + path;
    close();
    return false;
  }
  // scan: stop at the first record that is short, malformed or fails its checksum
  int64_t off = kFileHead;
  std::vector<unsigned char> buf;
  while (off + (int64_t)kHead + 8 <= file_bytes_) {
    RecHead rh;
    if (!read_at(fd_, &rh, kHead, off)) break;
    if (rh.magic != kRecMagic || rh.has_beta > 1 || rh.zero != 0 || rh.nl < 1 || rh.nl > 3 || rh.ntri < 0 ||
        rh.ntri > (1 << 24) || rh.d < 0 || rh.d > 3 * 128 || rh.np < 1)
      break;
    const int64_t pay = journal_payload_doubles(rh.nl, rh.ntri, rh.d, (int)rh.has_beta) * 8;
    const int64_t total = (int64_t)kHead + pay + 8;
    if (off + total > file_bytes_) break;
    buf.resize((size_t)total);
    if (!read_at(fd_, buf.data(), (size_t)total, off)) break;
    uint64_t sum;
    std::memcpy(&sum, buf.data() + kHead + pay, 8);
    if (fnv1a64(buf.data(), (size_t)(kHead + pay)) != sum) break;
    recs_.push_back({rh.key, rh.hash, rh.np, rh.nl, rh.ntri, rh.d, (int)rh.has_beta, off});
    off += total;
  }
  valid_bytes_ = off;
  // a torn tail (a writer killed mid-record) is cut off before anything is appended
  if (create && valid_bytes_ < file_bytes_) {
    if (::ftruncate(fd_, valid_bytes_) != 0) {
      err = sys_err("cannot cut the torn tail of journal", path);
      close();
      return false;
    }
    file_bytes_ = valid_bytes_;
  }
  return true;
}

// The last record of (key, hash) wins: a mock recorded without beta and run
// again for a caller that asks for beta is appended once more, with beta.
const JournalRecord* Journal::find(uint64_t key, uint64_t hash) const {
  for (auto it = recs_.rbegin(); it != recs_.rend(); ++it)
    if (it->key == key && it->hash == hash) return &*it;
  return nullptr;
}

bool Journal::read(const JournalRecord& r, double* B, double* alpha, double* beta, std::string& err) const {
  int64_t off = r.offset + (int64_t)kHead;
  const size_t nb = (size_t)r.nl * r.ntri * 8, nd = (size_t)r.d * 8;
  bool ok = read_at(fd_, B, nb, off);
  off += nb;
  ok = ok && read_at(fd_, alpha, nd, off);
  off += nd;
  if (beta && r.has_beta) ok = ok && read_at(fd_, beta, nd, off);
  if (!ok) err = sys_err("cannot read journal record of", path_);
  return ok;
}

bool Journal::append(uint64_t key, uint64_t hash, int64_t np, int nl, int ntri, int d, const double* B,
                     const double* alpha, const double* beta, bool sync, std::string& err) {
  RecHead rh{kRecMagic, beta ? 1u : 0u, key, hash, np, nl, ntri, d, 0};
  const int64_t pay = journal_payload_doubles(nl, ntri, d, beta ? 1 : 0) * 8;
  std::vector<unsigned char> buf((size_t)(kHead + pay + 8));
  unsigned char* p = buf.data();
  std::memcpy(p, &rh, kHead);
  p += kHead;
  std::memcpy(p, B, (size_t)nl * ntri * 8);
  p += (size_t)nl * ntri * 8;
  std::memcpy(p, alpha, (size_t)d * 8);
  p += (size_t)d * 8;
  if (beta) {
    std::memcpy(p, beta, (size_t)d * 8);
    p += (size_t)d * 8;
  }
  const uint64_t sum = fnv1a64(buf.data(), (size_t)(kHead + pay));
  std::memcpy(p, &sum, 8);
  if (!write_at(fd_, buf.data(), buf.size(), valid_bytes_) || (sync && ::fdatasync(fd_) != 0)) {
    err = sys_err("cannot append to journal", path_);
    return false;
  }
  recs_.push_back({key, hash, np, nl, ntri, d, beta ? 1 : 0, valid_bytes_});
  valid_bytes_ += (int64_t)buf.size();
  file_bytes_ = valid_bytes_;
  return true;
}

}  // namespace bsp
