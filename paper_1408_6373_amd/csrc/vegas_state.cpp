// vegas_state.cpp -- a Vegas integral's state file (checkpoint and resume).
//
// The Vegas prototype of Sect. 3.2.2 takes a state file.  Here it is written
// after every iteration; a later call with the same settings continues from
// it.  Because iteration t's points depend only on (seed, stream, t, i), a
// resumed run samples exactly the points the uninterrupted run would have.
#include "vegas_state.h"

#include <cstdio>
#include <cstring>

namespace ccuba {

namespace {

constexpr char kMagic[8] = {'C', 'C', 'U', 'B', 'A', 'V', 'S', '1'};

// the settings a state belongs to (budget and tolerances may change between
// the calls that share a file)
struct Header {
  char magic[8];
  int version;
  int state_bytes;  // sizeof(VState) of the writer
  int ndim, nbins, family, prec, flags;
  unsigned int sid;
  unsigned long long seed;
  long long nstart, nincrease;
  double a[kMaxDim], u[kMaxDim];
  int T;  // iterations in the history
  int pad;
};

Header header_of(const VegasSpec &sp, int T) {
  Header h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, sizeof(kMagic));
  h.version = 2;  // 2: the state holds the shift of the sums
  h.state_bytes = (int)sizeof(VState);
  h.ndim = sp.ndim;
  h.nbins = sp.nbins;
  h.family = sp.family;
  h.prec = sp.prec;
  h.flags = sp.flags;
  h.sid = sp.sid;
  h.seed = sp.seed;
  h.nstart = sp.nstart;
  h.nincrease = sp.nincrease;
  for (int j = 0; j < sp.ndim; ++j) {
    h.a[j] = sp.a[j];
    h.u[j] = sp.u[j];
  }
  h.T = T;
  return h;
}

}  // namespace

int state_read(const char *path, const VegasSpec &sp, StateFile &out) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return 1;
  Header h, want = header_of(sp, 0);
  bool ok = std::fread(&h, sizeof(h), 1, f) == 1;
  want.T = h.T;
  ok = ok && std::memcmp(&h, &want, sizeof(h)) == 0 && h.T >= 0 && h.T < (1 << 24);
  const size_t row = (size_t)sp.ndim * (sp.nbins + 1);
  if (ok) {
    out.grid.resize(row);
    out.I.resize(h.T);
    out.var.resize(h.T);
    ok = std::fread(&out.st, sizeof(VState), 1, f) == 1 &&
         std::fread(out.grid.data(), sizeof(double), row, f) == row &&
         std::fread(out.I.data(), sizeof(double), h.T, f) == (size_t)h.T &&
         std::fread(out.var.data(), sizeof(double), h.T, f) == (size_t)h.T &&
         out.st.T == h.T;
  }
  std::fclose(f);
  return ok ? 0 : CCUBA_EINVAL;
}

int state_write(const char *path, const VegasSpec &sp, const StateFile &sf) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return CCUBA_EINVAL;
  const int T = sf.st.T;
  const Header h = header_of(sp, T);
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
            std::fwrite(&sf.st, sizeof(VState), 1, f) == 1 &&
            std::fwrite(sf.grid.data(), sizeof(double), sf.grid.size(), f) == sf.grid.size() &&
            std::fwrite(sf.I.data(), sizeof(double), T, f) == (size_t)T &&
            std::fwrite(sf.var.data(), sizeof(double), T, f) == (size_t)T;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return CCUBA_EINVAL;
  }
  return CCUBA_OK;
}

}  // namespace ccuba
