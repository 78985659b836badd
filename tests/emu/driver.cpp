// Test driver for the CPU-emulated xs21 library (test infrastructure only).
//
// Reads a plain-text spec, runs the C-ABI on emulated "device" memory
// (malloc, so AddressSanitizer sees out-of-bounds accesses), and writes raw
// little-endian outputs for the Python tests to compare with the oracle.
//
// Spec lines:
//   storage f32|bf16|f64
//   max_walkers W
//   max_plain R
//   box <file> <dtype f32|f64> <n> <L> <z> <nbins>
//   walker <zeta> <r_mfp> <t_vir>
//   walker2 <zeta0> <r_mfp> <t_feed> <alpha> <beta>
//   out <dir>
//   prepare
//   batch                      -> batch_pk.bin [nw][nb][nbmax] f64, batch_xhi.bin [nw][nb] f64
//   plain <box> <walker> [radii file|-]  -> plain_b{b}_w{w}_{xhi,dtb,pk,xm}.bin
//   materialize <box> <walker> -> mat_b{b}_w{w}_{xhi,dtb}.bin
//   batch2 <nbmax> [tag]       -> batch2<tag>_{pk,xhi}.bin for the walker2 list
//   materialize2 <box> <walker2> -> mat2_b{b}_w{w}_{xhi,dtb}.bin
//   mcmc <dim> <a> <nw> <steps> <lo/hi file> <x file> <u file> <tag>
//        -> mcmc<tag>_x.bin [steps+1][nw][dim], _lp.bin [steps+1][nw], _acc.bin [steps][nw] int32
//   batch_fields <nbmax> <walker> <box> -> batchf_{pk,xhi,fx,fd}.bin (fields of that walker on that box)
//   erfc <file> <count>        -> erfc.bin: the FP32 erfc of the ionisation pass at count floats
//   tuning <n> <ion> <pipe> <bins> <flag> <group>  -> xs21_set_tuning for grid size n
//   autotune <reps> <cache> <tag> -> tune<tag>.bin: int32 [ion, pipe, bins, flag, group, from_cache]
//   smoothed <box> <index>     -> sm_b{b}_j{j}.bin
//   pk <box> <field file>      -> fpk_b{b}.bin
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <list>
#include <string>
#include <vector>

#include "xs21.h"

static std::vector<char> read_file(const std::string& p) {
  std::ifstream f(p, std::ios::binary);
  if (!f) {
    std::fprintf(stderr, "cannot read %s\n", p.c_str());
    std::exit(2);
  }
  return std::vector<char>((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
}

static void write_file(const std::string& p, const void* d, size_t n) {
  std::ofstream f(p, std::ios::binary);
  f.write(static_cast<const char*>(d), static_cast<std::streamsize>(n));
}

#define CHECK(call)                                                                   \
  do {                                                                                \
    xs21_status s_ = (call);                                                          \
    if (s_ != XS21_OK) {                                                              \
      std::fprintf(stderr, "%s failed: %d %s\n", #call, (int)s_, xs21_last_error()); \
      return 3;                                                                       \
    }                                                                                 \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 2) return 1;
  std::ifstream spec(argv[1]);
  xs21_physics phys;
  xs21_physics_default(&phys);
  xs21_dtype storage = XS21_F32;
  int max_walkers = 8, max_plain = 40;
  std::vector<xs21_walker> walkers;
  std::vector<xs21_walker2> walkers2;
  std::vector<int> box_dtype, box_n;
  std::vector<std::vector<char>> box_data;
  std::list<std::vector<char>> staged;  // inputs of queued device work, kept to the end
  std::vector<double> last_pk;           // P(k) of the last batch (device memory is host memory here)
  std::string out = ".";
  xs21_ctx* ctx = nullptr;
  void* ws = nullptr;
  std::string line;
  while (std::getline(spec, line)) {
    std::istringstream is(line);
    std::string cmd;
    if (!(is >> cmd) || cmd[0] == '#') continue;
    if (cmd == "phys") {
      std::string key;
      double v;
      is >> key >> v;
      if (key == "pk_amp") phys.pk_amp = v;
      else if (key == "ladder_top") phys.ladder_top = v;
      else if (key == "radius_step") phys.radius_step = v;
      else if (key == "mmin_form") phys.mmin_form = static_cast<int>(v);
      else if (key == "velocity") phys.velocity = static_cast<int>(v);
      else if (key == "dvdr_max") phys.dvdr_max = v;
    } else if (cmd == "storage") {
      std::string s;
      is >> s;
      storage = s == "bf16" ? XS21_BF16 : (s == "f64" ? XS21_F64 : XS21_F32);
    } else if (cmd == "max_walkers") {
      is >> max_walkers;
    } else if (cmd == "max_plain") {
      is >> max_plain;
    } else if (cmd == "out") {
      is >> out;
    } else if (cmd == "walker") {
      xs21_walker w;
      is >> w.zeta >> w.r_mfp >> w.t_vir;
      walkers.push_back(w);
    } else if (cmd == "walker2") {
      xs21_walker2 w;
      is >> w.zeta0 >> w.r_mfp >> w.t_feed >> w.alpha >> w.beta;
      walkers2.push_back(w);
    } else if (cmd == "batch2") {
      const int nb = static_cast<int>(box_n.size());
      std::vector<xs21_box> bx(nb);
      for (int i = 0; i < nb; ++i) bx[i] = i;
      int nbmax = 0;
      std::string tag;
      is >> nbmax >> tag;
      const int nw = static_cast<int>(walkers2.size());
      std::vector<double> pk(static_cast<size_t>(nw) * nb * nbmax, -1.0), xm(static_cast<size_t>(nw) * nb, -1.0);
      CHECK(xs21_eval_batch2(ctx, bx.data(), nb, walkers2.data(), nw, pk.data(), xm.data()));
      CHECK(xs21_sync(ctx));
      write_file(out + "/batch2" + tag + "_pk.bin", pk.data(), pk.size() * 8);
      write_file(out + "/batch2" + tag + "_xhi.bin", xm.data(), xm.size() * 8);
    } else if (cmd == "batch_fields") {
      const int nb = static_cast<int>(box_n.size());
      std::vector<xs21_box> bx(nb);
      for (int i = 0; i < nb; ++i) bx[i] = i;
      int nbmax = 0, fw = 0, fb = 0;
      is >> nbmax >> fw >> fb;
      const int nw = static_cast<int>(walkers.size());
      const size_t cells = static_cast<size_t>(box_n[fb]) * box_n[fb] * box_n[fb];
      const size_t rs = box_dtype[fb] == XS21_F64 ? 8 : 4;
      std::vector<double> pk(static_cast<size_t>(nw) * nb * nbmax, -1.0), xm(static_cast<size_t>(nw) * nb, -1.0);
      std::vector<char> fx(cells * rs), fd(cells * rs);
      CHECK(xs21_eval_batch_fields(ctx, bx.data(), nb, walkers.data(), nw, pk.data(), xm.data(), fw, fb, fx.data(),
                                   fd.data()));
      CHECK(xs21_sync(ctx));
      write_file(out + "/batchf_pk.bin", pk.data(), pk.size() * 8);
      write_file(out + "/batchf_xhi.bin", xm.data(), xm.size() * 8);
      write_file(out + "/batchf_fx.bin", fx.data(), fx.size());
      write_file(out + "/batchf_fd.bin", fd.data(), fd.size());
    } else if (cmd == "tuning") {
      int n;
      xs21_tuning t;
      is >> n >> t.ion_blocks >> t.pipe_blocks >> t.bins_blocks >> t.flag_test >> t.group;
      CHECK(xs21_set_tuning(ctx, n, &t));
    } else if (cmd == "autotune") {
      int reps;
      std::string cache, tag;
      is >> reps >> cache >> tag;
      const int nb = static_cast<int>(box_n.size());
      std::vector<xs21_box> bx(nb);
      for (int i = 0; i < nb; ++i) bx[i] = i;
      xs21_tuning t;
      double ms = 0;
      int cached = -1;
      CHECK(xs21_autotune(ctx, bx.data(), nb, walkers.data(), static_cast<int>(walkers.size()), reps, cache.c_str(),
                          &t, &ms, &cached));
      const int32_t v[6] = {t.ion_blocks, t.pipe_blocks, t.bins_blocks, t.flag_test, t.group, cached};
      write_file(out + "/tune" + tag + ".bin", v, sizeof v);
    } else if (cmd == "erfc") {
      std::string f;
      long count = 0;
      is >> f >> count;
      auto xv = read_file(f);
      std::vector<float> y(count);
      if (!ctx) CHECK(xs21_create(&ctx, 0, nullptr, &phys));
      CHECK(xs21_erfc_f32(ctx, reinterpret_cast<const float*>(xv.data()), y.data(), count));
      CHECK(xs21_sync(ctx));
      write_file(out + "/erfc.bin", y.data(), y.size() * 4);
    } else if (cmd == "materialize2") {
      int b, w;
      is >> b >> w;
      const size_t cells = static_cast<size_t>(box_n[b]) * box_n[b] * box_n[b];
      const size_t rs = box_dtype[b] == XS21_F64 ? 8 : 4;
      std::vector<char> xhi(cells * rs), dtb(cells * rs);
      CHECK(xs21_materialize2(ctx, b, &walkers2[w], xhi.data(), dtb.data()));
      CHECK(xs21_sync(ctx));
      char pre[512];
      std::snprintf(pre, sizeof pre, "%s/mat2_b%d_w%d_", out.c_str(), b, w);
      write_file(std::string(pre) + "xhi.bin", xhi.data(), xhi.size());
      write_file(std::string(pre) + "dtb.bin", dtb.data(), dtb.size());
    } else if (cmd == "mcmc") {
      int dim, nw, steps;
      double a;
      std::string bf, xf, uf, tag;
      is >> dim >> a >> nw >> steps >> bf >> xf >> uf >> tag;
      xs21_sampler sp{};
      sp.dim = dim;
      sp.a = a;
      auto bounds = read_file(bf);
      for (int c = 0; c < dim; ++c) {
        sp.lo[c] = reinterpret_cast<const double*>(bounds.data())[c];
        sp.hi[c] = reinterpret_cast<const double*>(bounds.data())[dim + c];
      }
      auto xv = read_file(xf);
      auto uv = read_file(uf);
      std::vector<double> x(reinterpret_cast<const double*>(xv.data()),
                            reinterpret_cast<const double*>(xv.data()) + static_cast<size_t>(nw) * dim);
      std::vector<double> lp(nw);
      std::vector<int32_t> acc(nw);
      std::vector<double> xs, lps;
      std::vector<int32_t> accs;
      const int nb = static_cast<int>(box_n.size());
      std::vector<xs21_box> bx(nb);
      for (int i = 0; i < nb; ++i) bx[i] = i;
      CHECK(xs21_mcmc_lnprob(ctx, bx.data(), nb, &sp, x.data(), nw, lp.data()));
      CHECK(xs21_sync(ctx));
      xs.insert(xs.end(), x.begin(), x.end());
      lps.insert(lps.end(), lp.begin(), lp.end());
      for (int t = 0; t < steps; ++t) {
        const double* u = reinterpret_cast<const double*>(uv.data()) + static_cast<size_t>(t) * nw * 3;
        CHECK(xs21_mcmc_step(ctx, bx.data(), nb, &sp, x.data(), lp.data(), nw, u, acc.data()));
        CHECK(xs21_sync(ctx));
        xs.insert(xs.end(), x.begin(), x.end());
        lps.insert(lps.end(), lp.begin(), lp.end());
        accs.insert(accs.end(), acc.begin(), acc.end());
      }
      write_file(out + "/mcmc" + tag + "_x.bin", xs.data(), xs.size() * 8);
      write_file(out + "/mcmc" + tag + "_lp.bin", lps.data(), lps.size() * 8);
      write_file(out + "/mcmc" + tag + "_acc.bin", accs.data(), accs.size() * 4);
    } else if (cmd == "box") {
      if (!ctx) CHECK(xs21_create(&ctx, 0, nullptr, &phys));
      std::string file, dt;
      int n, nb;
      double L, z;
      is >> file >> dt >> n >> L >> z >> nb;
      box_data.push_back(read_file(file));
      const xs21_dtype d = dt == "f64" ? XS21_F64 : XS21_F32;
      box_dtype.push_back(d);
      box_n.push_back(n);
      xs21_box h;
      CHECK(xs21_add_box(ctx, box_data.back().data(), 0, d, n, L, z, nb, &h));
    } else if (cmd == "prepare") {
      size_t bytes = 0;
      CHECK(xs21_workspace_size(ctx, storage, max_walkers, max_plain, &bytes));
      ws = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
      // poison: NaN bytes so that reads of never-written workspace show up
      std::memset(ws, 0xff, bytes);
      CHECK(xs21_prepare(ctx, ws, bytes, storage, max_walkers, max_plain));
      std::printf("workspace %zu\n", bytes);
    } else if (cmd == "batch") {
      // batch <nbmax> [tag]: every walker on every box, outputs batch<tag>_*.bin
      const int nb = static_cast<int>(box_n.size());
      std::vector<xs21_box> bx(nb);
      for (int i = 0; i < nb; ++i) bx[i] = i;
      int nbmax = 0;
      std::string tag;
      is >> nbmax >> tag;
      const int nw = static_cast<int>(walkers.size());
      std::vector<double> pk(static_cast<size_t>(nw) * nb * nbmax, -1.0), xm(static_cast<size_t>(nw) * nb, -1.0);
      CHECK(xs21_eval_batch(ctx, bx.data(), nb, walkers.data(), nw, pk.data(), xm.data()));
      CHECK(xs21_sync(ctx));
      write_file(out + "/batch" + tag + "_pk.bin", pk.data(), pk.size() * 8);
      write_file(out + "/batch" + tag + "_xhi.bin", xm.data(), xm.size() * 8);
      last_pk = pk;
    } else if (cmd == "mock") {
      // mock <box> <mock file> <noise file|-> <model_err> <k_lo> <k_hi>
      int b;
      std::string mf, nf;
      double me, klo, khi;
      is >> b >> mf >> nf >> me >> klo >> khi;
      auto m = read_file(mf);
      std::vector<char> nz;
      if (nf != "-") nz = read_file(nf);
      CHECK(xs21_set_mock(ctx, b, reinterpret_cast<const double*>(m.data()),
                          nz.empty() ? nullptr : reinterpret_cast<const double*>(nz.data()), me, klo, khi));
    } else if (cmd == "chi2") {
      // chi2 [tag]: chi^2 of every walker over all boxes from the last batch's P(k)
      std::string tag;
      is >> tag;
      const int nb = static_cast<int>(box_n.size());
      std::vector<xs21_box> bx(nb);
      for (int i = 0; i < nb; ++i) bx[i] = i;
      const int nw = static_cast<int>(walkers.size());
      std::vector<double> c2(nw, -1.0);
      CHECK(xs21_chi2(ctx, bx.data(), nb, last_pk.data(), nw, c2.data()));
      CHECK(xs21_sync(ctx));
      write_file(out + "/chi2" + tag + ".bin", c2.data(), c2.size() * 8);
    } else if (cmd == "resmooth") {
      // resmooth <box> <file|->: new density (same dtype and size) or the current one
      int b;
      std::string ff;
      is >> b >> ff;
      const void* src = nullptr;
      if (ff != "-") {
        staged.push_back(read_file(ff));
        src = staged.back().data();
      }
      CHECK(xs21_resmooth(ctx, b, src));
    } else if (cmd == "plain") {
      int b, w;
      std::string rf;
      is >> b >> w >> rf;
      std::vector<double> radii;
      if (!rf.empty() && rf != "-") {
        auto d = read_file(rf);
        radii.resize(d.size() / 8);
        std::memcpy(radii.data(), d.data(), d.size());
      }
      const size_t cells = static_cast<size_t>(box_n[b]) * box_n[b] * box_n[b];
      const size_t rs = box_dtype[b] == XS21_F64 ? 8 : 4;
      std::vector<char> xhi(cells * rs), dtb(cells * rs);
      double pk[64], km[64], cnt[64], xm = -1;
      CHECK(xs21_eval(ctx, b, &walkers[w], radii.empty() ? nullptr : radii.data(), static_cast<int>(radii.size()),
                      xhi.data(), dtb.data(), pk, km, cnt, &xm));
      char pre[512];
      std::snprintf(pre, sizeof pre, "%s/plain_b%d_w%d_", out.c_str(), b, w);
      write_file(std::string(pre) + "xhi.bin", xhi.data(), xhi.size());
      write_file(std::string(pre) + "dtb.bin", dtb.data(), dtb.size());
      write_file(std::string(pre) + "pk.bin", pk, 64 * 8);
      write_file(std::string(pre) + "km.bin", km, 64 * 8);
      write_file(std::string(pre) + "cnt.bin", cnt, 64 * 8);
      write_file(std::string(pre) + "xm.bin", &xm, 8);
    } else if (cmd == "materialize") {
      int b, w;
      is >> b >> w;
      const size_t cells = static_cast<size_t>(box_n[b]) * box_n[b] * box_n[b];
      const size_t rs = box_dtype[b] == XS21_F64 ? 8 : 4;
      std::vector<char> xhi(cells * rs), dtb(cells * rs);
      CHECK(xs21_materialize(ctx, b, &walkers[w], xhi.data(), dtb.data()));
      CHECK(xs21_sync(ctx));
      char pre[512];
      std::snprintf(pre, sizeof pre, "%s/mat_b%d_w%d_", out.c_str(), b, w);
      write_file(std::string(pre) + "xhi.bin", xhi.data(), xhi.size());
      write_file(std::string(pre) + "dtb.bin", dtb.data(), dtb.size());
    } else if (cmd == "smoothed") {
      int b, j;
      is >> b >> j;
      const size_t cells = static_cast<size_t>(box_n[b]) * box_n[b] * box_n[b];
      const size_t rs = box_dtype[b] == XS21_F64 ? 8 : 4;
      std::vector<char> o(cells * rs);
      CHECK(xs21_smoothed(ctx, b, j, o.data()));
      CHECK(xs21_sync(ctx));
      char pre[512];
      std::snprintf(pre, sizeof pre, "%s/sm_b%d_j%d.bin", out.c_str(), b, j);
      write_file(pre, o.data(), o.size());
    } else if (cmd == "pk") {
      int b;
      std::string ff;
      is >> b >> ff;
      auto field = read_file(ff);
      double pk[64];
      CHECK(xs21_power_spectrum(ctx, b, field.data(), pk));
      char pre[512];
      std::snprintf(pre, sizeof pre, "%s/fpk_b%d.bin", out.c_str(), b);
      write_file(pre, pk, 64 * 8);
    } else {
      std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
      return 1;
    }
  }
  xs21_destroy(ctx);
  std::free(ws);
  return 0;
}
