// ULV-like factorization (Alg. 3) and solve (Alg. 4, App. A) of an HSS
// handle whose U generators have the ID structure U = Pi [I; E] (Sec. 2.4).
//
// Factorization, level by level over heights (children first):
//  * D_tau = D at a leaf; at an inner node
//    D_tau = [Dt_a, B_ab Vt_{b;b}^T ; B_ba Vt_{a;b}^T, Dt_b];
//  * Omega = [-E I; I 0] Pi^T turns U into [0; I]:
//    W_t = D_tau(rest) - E D_tau(J), W_b = D_tau(J);
//  * the LQ factorization W_t = [L 0] Q is a Householder QR of W_t^T.  It is
//    run once on Z = [W_t; Vh^T; W_b] (rows), factoring the first m-k rows and
//    carrying the others along, so one pass also yields (Q Vh)^T and W_b Q^T
//    (Vh = V at a leaf, diag(Vt_{a;b}, Vt_{b;b}) V above);
//  * at the root, D_root is factored by LU with partial pivoting.
// Solve: bottom-up b_tau, Omega b_tau, y = L^{-1} bt_t, z = Vt_t^T y
// (+ V^T [z_a; z_b]); root LU solve; top-down x_a = Q_a^T [y_a; x_tau(top)].
// All arithmetic runs in the HIP kernels (batched GEMM, QR, ULV kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "hss_handle.h"
#include "hss_ulv_kernels.h"

using namespace hss;

namespace {

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return set_error(HSS_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define CHK(x)                     \
  do {                             \
    hss_status st_ = (x);          \
    if (st_ != HSS_OK) return st_; \
  } while (0)

inline Seg seg(const double* p, long long ld, const int* map = nullptr) {
  return Seg{p, nullptr, ld, INT_MAX, map};
}
inline SegOut out(double* p, long long ld, const int* map = nullptr) {
  return SegOut{p, nullptr, ld, INT_MAX, map};
}

// copy of an M x N block (K = 0 GEMM)
GemmDesc copy_desc(int M, int N, const Seg& src, const SegOut& dst) {
  GemmDesc g{};
  g.M = M;
  g.N = N;
  g.K = 0;
  g.C = src;
  g.D = dst;
  g.alpha = 1.0;
  g.beta = 1.0;
  return g;
}

int md_of(const Node& v) { return v.leaf() ? v.size() : v.mr; }

// Blocked triangular solve X <- T^{-1} X for a batch: lower (forward) or
// upper (backward) T of order n (ld ldt), X n x nrhs (ld ldx).
struct TriJob {
  const double* T;
  long long ldt;
  double* X;
  long long ldx;
  int n, nrhs;
};

hss_status tri_solve_batch(const std::vector<TriJob>& jobs, bool lower, bool unit, Staging& st,
                           hipStream_t s) {
  // right-looking: solve a diagonal block of 64, then update every row still
  // to come with it (inner dimension <= 64, all those rows in one product).
  // Taking the solved blocks into each new block instead (inner dimension
  // growing to n, a 64 x nrhs output) left a few workgroups to run ever
  // longer products: 10 to 50 us each in the root solve of an N=32768 matrix.
  int nmax = 0;
  for (const TriJob& j : jobs) nmax = std::max(nmax, j.n);
  const int nblk = (nmax + 63) / 64;
  std::vector<GemmDesc> gd;
  std::vector<TriDesc> td;
  for (int step = 0; step < nblk; ++step) {
    gd.clear();
    td.clear();
    for (const TriJob& j : jobs) {
      const int nb_j = (j.n + 63) / 64;
      if (step >= nb_j || j.nrhs <= 0) continue;
      const int b = lower ? step : nb_j - 1 - step;
      const int b0 = b * 64, b1 = std::min(j.n, b0 + 64);
      TriDesc t{};
      t.T = j.T + (long long)b0 * j.ldt + b0;
      t.ldt = j.ldt;
      t.X = j.X + (long long)b0 * j.ldx;
      t.ldx = j.ldx;
      t.nb = b1 - b0;
      t.nrhs = j.nrhs;
      t.lower = lower ? 1 : 0;
      t.unit = unit ? 1 : 0;
      td.push_back(t);
      // the rows still to come: below the block (lower) or above it (upper)
      const int r0 = lower ? b1 : 0, r1 = lower ? j.n : b0;
      if (r1 > r0) {
        GemmDesc g{};
        g.M = r1 - r0;
        g.N = j.nrhs;
        g.K = b1 - b0;
        g.A = j.T + (long long)r0 * j.ldt + b0;
        g.lda = j.ldt;
        g.B = seg(j.X + (long long)b0 * j.ldx, j.ldx);
        g.C = seg(j.X + (long long)r0 * j.ldx, j.ldx);
        g.D = out(j.X + (long long)r0 * j.ldx, j.ldx);
        g.alpha = -1.0;
        g.beta = 1.0;
        gd.push_back(g);
      }
    }
    HIPCHK(launch_tri_block(td.data(), (int)td.size(), st, s));
    HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), st, s));
  }
  return HSS_OK;
}

// v <- H_0 H_1 ... H_{r-1} v for every descriptor (H_i = I - tau_i u_i u_i^T,
// u_i in row i of Z), in the compact WY form: the reflectors in blocks of 64,
// H_{i0} ... H_{i0+kb-1} = I - Y_b T_b Y_b^T, applied from the last block as
// W = Y_b^T v, W = T_b W, v = v - Y_b W.  Y_b is zero above its block's first
// row, so every product starts there.  Every step is a batched GEMM over all
// descriptors, so a large problem spreads over the device.
hss_status apply_q_blocked(Handle& H, const std::vector<ReflDesc>& rd, hipStream_t s) {
  if (rd.empty()) return HSS_OK;
  for (const ReflDesc& d : rd)
    if (!d.transpose) return set_error(HSS_ERR_ARG, "apply_q_blocked: only the H_0 ... H_{r-1} v form");
  const size_t np = rd.size();
  // W1 = Y_b^T v has at most 64 x nrhs entries but an inner dimension of up
  // to m: above 2 KC it is split into KC-row parts, each its own product,
  // whose results sum_partials adds in order (one workgroup per output tile
  // took 100-175 us on the top levels of an N=32768 solve)
  constexpr int KC = 256;
  std::vector<long long> oy(np), ow1(np), ow2(np), opt(np);
  std::vector<int> nb(np), ob(np);
  long long tot = 0;
  int nbtot = 0, nbmax = 0, rmax = 0, mmax = 0;
  for (size_t p = 0; p < np; ++p) {
    const ReflDesc& d = rd[p];
    oy[p] = tot;
    tot += (long long)d.m * d.r;
    ow1[p] = tot;
    tot += 64LL * d.nrhs;
    ow2[p] = tot;
    tot += 64LL * d.nrhs;
    opt[p] = tot;
    if (d.m > 2 * KC) tot += (long long)((d.m + KC - 1) / KC) * 64 * d.nrhs;
    nb[p] = (d.r + 63) / 64;
    ob[p] = nbtot;
    nbtot += nb[p];
    nbmax = std::max(nbmax, nb[p]);
    rmax = std::max(rmax, d.r);
    mmax = std::max(mmax, d.m);
  }
  // Y and T made by the factor (every descriptor has them) or here
  bool pre = true;
  for (const ReflDesc& d : rd) pre = pre && d.Y && d.T;
  const long long og = tot;
  if (!pre) tot += 2LL * nbtot * 64 * 64;
  double* ws = static_cast<double*>(H.work_misc.ensure((size_t)tot * 8 + 8, s));
  if (!ws) return set_error(HSS_ERR_ALLOC, "reflector workspace");
  auto Y = [&](size_t p) -> const double* { return pre ? rd[p].Y : ws + oy[p]; };
  auto Tb = [&](size_t p, int b) -> const double* {
    return pre ? rd[p].T + (long long)b * 64 * 64 : ws + og + (long long)(nbtot + ob[p] + b) * 64 * 64;
  };
  if (!pre) {
    std::vector<ReflYDesc> yd(np);
    for (size_t p = 0; p < np; ++p) yd[p] = ReflYDesc{rd[p].Z, rd[p].ldz, ws + oy[p], rd[p].r, rd[p].m};
    HIPCHK(launch_refl_y(yd.data(), (int)np, rmax, mmax, H.staging, s));
    // G_b = Y_b^T Y_b, then T_b
    std::vector<GemmDesc> gd;
    std::vector<LarftDesc> ld;
    for (size_t p = 0; p < np; ++p) {
      const ReflDesc& d = rd[p];
      for (int b = 0; b < nb[p]; ++b) {
        const int i0 = 64 * b, kb = std::min(64, d.r - i0);
        const double* yb = Y(p) + (long long)i0 * d.r + i0;
        double* gb = ws + og + (long long)(ob[p] + b) * 64 * 64;
        GemmDesc g{};
        g.M = g.N = kb;
        g.K = d.m - i0;
        g.A = yb;
        g.lda = d.r;
        g.transA = 1;
        g.B = seg(yb, d.r);
        g.D = out(gb, 64);
        g.alpha = 1.0;
        g.beta = 0.0;
        gd.push_back(g);
        ld.push_back(LarftDesc{gb, d.tau + i0, const_cast<double*>(Tb(p, b)), kb});
      }
    }
    HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
    HIPCHK(launch_larft(ld.data(), (int)ld.size(), H.staging, s));
  }
  for (int step = 0; step < nbmax; ++step) {
    std::vector<GemmDesc> g1, g2, g3;
    std::vector<SumDesc> sums;
    for (size_t p = 0; p < np; ++p) {
      if (step >= nb[p]) continue;
      const ReflDesc& d = rd[p];
      const int b = nb[p] - 1 - step;
      const int i0 = 64 * b, kb = std::min(64, d.r - i0);
      const double* yb = Y(p) + (long long)i0 * d.r + i0;
      double* vb = d.V + (long long)i0 * d.ldv;
      double* w1 = ws + ow1[p];
      double* w2 = ws + ow2[p];
      const int K = d.m - i0;
      const int parts = K > 2 * KC ? (K + KC - 1) / KC : 1;
      double* pt = ws + opt[p];
      for (int q = 0; q < parts; ++q) {  // W1 = Y_b^T v, or its parts
        const int k0 = q * KC;
        GemmDesc g{};
        g.M = kb;
        g.N = d.nrhs;
        g.K = parts > 1 ? std::min(KC, K - k0) : K;
        g.A = yb + (long long)k0 * d.r;
        g.lda = d.r;
        g.transA = 1;
        g.B = seg(vb + (long long)k0 * d.ldv, d.ldv);
        g.D = out(parts > 1 ? pt + (long long)q * kb * d.nrhs : w1, d.nrhs);
        g.alpha = 1.0;
        g.beta = 0.0;
        g1.push_back(g);
      }
      if (parts > 1) sums.push_back(SumDesc{pt, (long long)kb * d.nrhs, parts, kb, d.nrhs, w1, d.nrhs});
      GemmDesc t{};  // W2 = T_b W1
      t.M = kb;
      t.N = d.nrhs;
      t.K = kb;
      t.A = Tb(p, b);
      t.lda = 64;
      t.B = seg(w1, d.nrhs);
      t.D = out(w2, d.nrhs);
      t.alpha = 1.0;
      t.beta = 0.0;
      g2.push_back(t);
      GemmDesc u{};  // v = v - Y_b W2
      u.M = d.m - i0;
      u.N = d.nrhs;
      u.K = kb;
      u.A = yb;
      u.lda = d.r;
      u.B = seg(w2, d.nrhs);
      u.C = seg(vb, d.ldv);
      u.D = out(vb, d.ldv);
      u.alpha = -1.0;
      u.beta = 1.0;
      g3.push_back(u);
    }
    HIPCHK(launch_gemm_batched(g1.data(), (int)g1.size(), H.staging, s));
    HIPCHK(launch_sum_partials(sums.data(), (int)sums.size(), H.staging, s));
    HIPCHK(launch_gemm_batched(g2.data(), (int)g2.size(), H.staging, s));
    HIPCHK(launch_gemm_batched(g3.data(), (int)g3.size(), H.staging, s));
  }
  return HSS_OK;
}

// The 4 blocks of D_tau for inner node t into Dm (ld md).
void merged_D(const Handle& H, int t, double* Dm, std::vector<GemmDesc>& gd) {
  const Node& v = H.nodes[t];
  const Node& a = H.nodes[v.left];
  const Node& b = H.nodes[v.right];
  const int md = a.kr + b.kr;
  const int ma = md_of(a), mb = md_of(b);
  const int ra = ma - a.kr, rb = mb - b.kr;
  // Dt_a, Dt_b: rows r+kc.. of Z, columns r..
  if (a.kr) gd.push_back(copy_desc(a.kr, a.kr, seg(a.Z + (long long)(ra + a.kc) * ma + ra, ma), out(Dm, md)));
  if (b.kr)
    gd.push_back(copy_desc(b.kr, b.kr, seg(b.Z + (long long)(rb + b.kc) * mb + rb, mb),
                           out(Dm + (long long)a.kr * md + a.kr, md)));
  // B_ab Vt_{b;b}^T: Vt_{b;b}^T = rows r_b..r_b+kc_b of Z_b, columns r_b..
  GemmDesc g{};
  g.M = a.kr;
  g.N = b.kr;
  g.K = b.kc;
  g.A = v.B12;
  g.lda = b.kc;
  g.B = seg(b.Z + (long long)rb * mb + rb, mb);
  g.D = out(Dm + a.kr, md);
  g.alpha = 1.0;
  g.beta = 0.0;
  if (g.M && g.N) gd.push_back(g);
  g.M = b.kr;
  g.N = a.kr;
  g.K = a.kc;
  g.A = v.B21;
  g.lda = a.kc;
  g.B = seg(a.Z + (long long)ra * ma + ra, ma);
  g.D = out(Dm + (long long)a.kr * md, md);
  if (g.M && g.N) gd.push_back(g);
}

// Once per factorization: every node's reflectors as a dense Y and the
// triangular factors T of its blocks of 64 (compact WY), which every solve
// applies (they depend on the factors only).
hss_status prepare_q(Handle& H, hipStream_t s) {
  std::vector<Node>& nd = H.nodes;
  std::vector<ReflYDesc> yd;
  std::vector<GemmDesc> gd;
  std::vector<LarftDesc> ld;
  long long gtot = 0;
  int rmax = 0, mmax = 0;
  for (size_t t = 1; t < nd.size(); ++t) {
    Node& u = nd[t];
    const int md = md_of(u), r = md - u.kr;
    if (r <= 0) continue;
    const int nb = (r + 63) / 64;
    u.Yq = static_cast<double*>(H.gen->alloc((size_t)md * r * 8));
    u.Tq = static_cast<double*>(H.gen->alloc((size_t)nb * 64 * 64 * 8));
    if (!u.Yq || !u.Tq) return set_error(HSS_ERR_ALLOC, "ULV reflector blocks");
    yd.push_back(ReflYDesc{u.Z, md, u.Yq, r, md});
    rmax = std::max(rmax, r);
    mmax = std::max(mmax, md);
    gtot += (long long)nb * 64 * 64;
  }
  if (yd.empty()) return HSS_OK;
  double* G = static_cast<double*>(H.work_misc.ensure((size_t)gtot * 8 + 8, s));
  if (!G) return set_error(HSS_ERR_ALLOC, "reflector workspace");
  HIPCHK(launch_refl_y(yd.data(), (int)yd.size(), rmax, mmax, H.staging, s));
  long long go = 0;
  for (size_t t = 1; t < nd.size(); ++t) {
    const Node& u = nd[t];
    const int md = md_of(u), r = md - u.kr;
    if (r <= 0) continue;
    for (int b = 0; b < (r + 63) / 64; ++b) {  // G_b = Y_b^T Y_b, then T_b
      const int i0 = 64 * b, kb = std::min(64, r - i0);
      const double* yb = u.Yq + (long long)i0 * r + i0;
      GemmDesc g{};
      g.M = g.N = kb;
      g.K = md - i0;
      g.A = yb;
      g.lda = r;
      g.transA = 1;
      g.B = seg(yb, r);
      g.D = out(G + go, 64);
      g.alpha = 1.0;
      g.beta = 0.0;
      gd.push_back(g);
      ld.push_back(LarftDesc{G + go, u.tau + i0, u.Tq + (long long)b * 64 * 64, kb});
      go += 64 * 64;
    }
  }
  HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
  HIPCHK(launch_larft(ld.data(), (int)ld.size(), H.staging, s));
  return HSS_OK;
}

hss_status factor_impl(Handle& H, hipStream_t s) {
  std::vector<Node>& nd = H.nodes;
  H.staging.stream = s;
  if (nd[0].leaf()) {
    const int n = (int)H.n;
    H.root_m = n;
    H.root_lu = static_cast<double*>(H.gen->alloc((size_t)n * n * 8));
    H.root_piv = static_cast<int*>(H.gen->alloc((size_t)n * 4));
    H.root_info = static_cast<int*>(H.gen->alloc(4));
    if (!H.root_lu || !H.root_piv || !H.root_info) return set_error(HSS_ERR_ALLOC, "root LU");
    HIPCHK(hipMemcpyAsync(H.root_lu, nd[0].D, (size_t)n * n * 8, hipMemcpyDeviceToDevice, s));
  } else {
    for (int h = 0; h < H.height; ++h) {
      const std::vector<int>& lvl = H.levels[h];
      // sizes and persistent buffers
      long long scratch = 0;
      for (int t : lvl) {
        Node& v = nd[t];
        const int md = md_of(v), r = md - v.kr;
        const long long rows = (long long)r + v.kc + v.kr;
        v.Z = static_cast<double*>(H.gen->alloc((size_t)std::max(1LL, rows * md) * 8));
        v.tau = static_cast<double*>(H.gen->alloc((size_t)std::max(1, r) * 8));
        if (!v.Z || !v.tau) return set_error(HSS_ERR_ALLOC, "ULV factors");
        if (!v.leaf()) {
          const Node& a = nd[v.left];
          const Node& b = nd[v.right];
          scratch += (long long)md * md + (long long)(a.kc + b.kc) * md;
        }
      }
      double* scr = nullptr;
      if (scratch > 0) {
        scr = static_cast<double*>(H.work_misc.ensure((size_t)scratch * 8, s));
        if (!scr) return set_error(HSS_ERR_ALLOC, "ULV scratch");
        HIPCHK(hipMemsetAsync(scr, 0, (size_t)scratch * 8, s));
      }
      // D_tau and X = diag(Vt_{a;b}^T, Vt_{b;b}^T) of the inner nodes
      std::vector<GemmDesc> gd;
      std::vector<double*> Dm(nd.size(), nullptr), X(nd.size(), nullptr);
      long long so = 0;
      for (int t : lvl) {
        Node& v = nd[t];
        if (v.leaf()) continue;
        const Node& a = nd[v.left];
        const Node& b = nd[v.right];
        const int md = md_of(v), ma = md_of(a), mb = md_of(b);
        const int ra = ma - a.kr, rb = mb - b.kr;
        Dm[t] = scr + so;
        so += (long long)md * md;
        X[t] = scr + so;
        so += (long long)(a.kc + b.kc) * md;
        merged_D(H, t, Dm[t], gd);
        if (a.kc && a.kr) gd.push_back(copy_desc(a.kc, a.kr, seg(a.Z + (long long)ra * ma + ra, ma), out(X[t], md)));
        if (b.kc && b.kr)
          gd.push_back(copy_desc(b.kc, b.kr, seg(b.Z + (long long)rb * mb + rb, mb),
                                 out(X[t] + (long long)a.kc * md + a.kr, md)));
      }
      HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
      // Z = [W_t; Vh^T; W_b]
      gd.clear();
      std::vector<VtLeafDesc> vl;
      int kmax_leaf = 0;
      for (int t : lvl) {
        Node& v = nd[t];
        const int md = md_of(v), k = v.kr, r = md - k;
        const double* Dt = v.leaf() ? v.D : Dm[t];
        GemmDesc g{};  // W_t = D(rest) - E D(J)
        g.M = r;
        g.N = md;
        g.K = k;
        g.A = v.Er;
        g.lda = k;
        g.B = seg(Dt, md, v.perm_r);
        g.C = seg(Dt, md, v.perm_r + k);
        g.D = out(v.Z, md);
        g.alpha = -1.0;
        g.beta = 1.0;
        if (r) gd.push_back(g);
        if (k) gd.push_back(copy_desc(k, md, seg(Dt, md, v.perm_r), out(v.Z + (long long)(r + v.kc) * md, md)));
        if (v.kc == 0) continue;
        if (v.leaf()) {
          VtLeafDesc x{v.Z + (long long)r * md, md, md, v.kc, v.perm_c, v.Ec};
          vl.push_back(x);
          kmax_leaf = std::max(kmax_leaf, v.kc);
        } else {  // Vh^T = V^T X = X(J) + E^T X(rest)
          GemmDesc e{};
          e.M = v.kc;
          e.N = md;
          e.K = v.mc - v.kc;
          e.A = v.Ec;
          e.lda = v.kc;
          e.transA = 1;
          e.B = seg(X[t], md, v.perm_c + v.kc);
          e.C = seg(X[t], md, v.perm_c);
          e.D = out(v.Z + (long long)r * md, md);
          e.alpha = 1.0;
          e.beta = 1.0;
          gd.push_back(e);
        }
      }
      HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
      HIPCHK(launch_vt_leaf(vl.data(), (int)vl.size(), kmax_leaf, H.staging, s));
      // LQ of W_t as a QR without pivoting of the first r rows of Z
      std::vector<IdProblem> pr;
      for (int t : lvl) {
        Node& v = nd[t];
        const int md = md_of(v), r = md - v.kr;
        if (r <= 0) continue;
        IdProblem p{};
        p.Y = v.Z;
        p.ldy = md;
        p.m = r + v.kc + v.kr;
        p.d = md;
        p.W = v.Z;
        p.ldw = md;
        p.kfail = -1;
        p.nfac = r;
        p.tau = v.tau;
        pr.push_back(p);
      }
      if (!pr.empty()) {
        const size_t wb = id_workspace_bytes(pr.data(), (int)pr.size());
        void* wk = H.work_id.ensure(wb, s);
        if (!wk) return set_error(HSS_ERR_ALLOC, "QR workspace");
        std::vector<int> kh(pr.size() + 2);
        HIPCHK(launch_id_factor(pr.data(), (int)pr.size(), 0.0, wk, H.work_id.cap, kh.data(), H.staging, s));
        HIPCHK(launch_qr_reflectors(pr.data(), (int)pr.size(), wk, H.staging, s));
      }
      HIPCHK(hipStreamSynchronize(s));
      H.staging.reset();
    }
    // root: D_root, then LU with partial pivoting
    Node& r = nd[0];
    const int m = nd[r.left].kr + nd[r.right].kr;
    H.root_m = m;
    H.root_lu = static_cast<double*>(H.gen->alloc((size_t)std::max(1, m * m) * 8));
    H.root_piv = static_cast<int*>(H.gen->alloc((size_t)std::max(1, m) * 4));
    H.root_info = static_cast<int*>(H.gen->alloc(4));
    if (!H.root_lu || !H.root_piv || !H.root_info) return set_error(HSS_ERR_ALLOC, "root LU");
    std::vector<GemmDesc> gd;
    merged_D(H, 0, H.root_lu, gd);
    HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
  }
  const int m = H.root_m;
  HIPCHK(hipMemsetAsync(H.root_info, 0, 4, s));
  // panels of 32 columns: the panel kernel updates its own trailing columns
  // in one workgroup, the GEMM below the rest on the whole device (N=32768
  // serving factor 65.9 ms with panels of 64, 62.2 with 32, 63.4 with 16)
  constexpr int PW = 32;
  for (int j0 = 0; j0 < m; j0 += PW) {
    const int nb = std::min(PW, m - j0), j1 = j0 + nb;
    HIPCHK(launch_lu_panel(H.root_lu, m, m, j0, nb, H.root_piv, H.root_info, s));
    HIPCHK(launch_lu_swap(H.root_lu, m, m, H.root_piv, j0, nb, j0, j1, s));
    if (j1 < m) {
      std::vector<TriJob> tj{TriJob{H.root_lu + (long long)j0 * m + j0, m, H.root_lu + (long long)j0 * m + j1,
                                    m, nb, m - j1}};
      CHK(tri_solve_batch(tj, true, true, H.staging, s));
      GemmDesc g{};
      g.M = g.N = m - j1;
      g.K = nb;
      g.A = H.root_lu + (long long)j1 * m + j0;
      g.lda = m;
      g.B = seg(H.root_lu + (long long)j0 * m + j1, m);
      g.C = seg(H.root_lu + (long long)j1 * m + j1, m);
      g.D = out(H.root_lu + (long long)j1 * m + j1, m);
      g.alpha = -1.0;
      g.beta = 1.0;
      HIPCHK(launch_gemm_batched(&g, 1, H.staging, s));
    }
  }
  CHK(prepare_q(H, s));
  int info = 0;
  HIPCHK(hipMemcpyAsync(&info, H.root_info, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  H.staging.reset();
  if (info != 0) return set_error(HSS_ERR_SINGULAR, "zero pivot in the root LU at column " + std::to_string(info));
  H.factored = true;
  return HSS_OK;
}

hss_status solve_impl(Handle& H, int nrhs, const double* b, long long ldb, double* x, long long ldx,
                      hipStream_t s) {
  std::vector<Node>& nd = H.nodes;
  H.staging.stream = s;
  const int m0 = H.root_m;
  // workspace: per node B (md x nrhs), T (md x nrhs), z (kc x nrhs), X (md x nrhs); root RB
  std::vector<long long> oB(nd.size()), oT(nd.size()), oz(nd.size()), oX(nd.size());
  long long tot = 0;
  for (size_t t = 1; t < nd.size(); ++t) {
    const long long md = md_of(nd[t]);
    oB[t] = tot;
    tot += md * nrhs;
    oT[t] = tot;
    tot += md * nrhs;
    oz[t] = tot;
    tot += (long long)nd[t].kc * nrhs;
    oX[t] = tot;
    tot += md * nrhs;
  }
  const long long oR = tot;
  tot += (long long)m0 * nrhs;
  double* ws = static_cast<double*>(H.work_mv.ensure((size_t)tot * 8 + 8, s));
  if (!ws) return set_error(HSS_ERR_ALLOC, "solve workspace");
  double* RB = ws + oR;
  auto Bp = [&](int t) { return ws + oB[t]; };
  auto Tp = [&](int t) { return ws + oT[t]; };
  auto Zp = [&](int t) { return ws + oz[t]; };
  auto Xp = [&](int t) { return ws + oX[t]; };
  std::vector<GemmDesc> gd;

  // right-hand side of an inner node (or the root) into dst:
  // [bt_{a;b} - W_{a;b} Q_{a;t}^T y_a - B_ab z_b ; bt_{b;b} - B_ba z_a - W_{b;b} Q_{b;t}^T y_b]
  auto rhs_inner = [&](int t, double* dst, std::vector<GemmDesc>& first, std::vector<GemmDesc>& second) {
    const Node& v = nd[t];
    const Node& a = nd[v.left];
    const Node& c = nd[v.right];
    const int ma = md_of(a), mc_ = md_of(c);
    const int ra = ma - a.kr, rc = mc_ - c.kr;
    GemmDesc g{};
    g.N = nrhs;
    g.alpha = -1.0;
    g.beta = 1.0;
    // top: bt_{a;b} - (W_b Q^T)_a[:, 0:ra] y_a
    g.M = a.kr;
    g.K = ra;
    g.A = a.Z + (long long)(ra + a.kc) * ma;
    g.lda = ma;
    g.B = seg(Tp(v.left), nrhs);
    g.C = seg(Tp(v.left) + (long long)ra * nrhs, nrhs);
    g.D = out(dst, nrhs);
    if (g.M) first.push_back(g);
    // bottom: bt_{b;b} - (W_b Q^T)_b[:, 0:rc] y_b
    g.M = c.kr;
    g.K = rc;
    g.A = c.Z + (long long)(rc + c.kc) * mc_;
    g.lda = mc_;
    g.B = seg(Tp(v.right), nrhs);
    g.C = seg(Tp(v.right) + (long long)rc * nrhs, nrhs);
    g.D = out(dst + (long long)a.kr * nrhs, nrhs);
    if (g.M) first.push_back(g);
    // - B_ab z_b, - B_ba z_a
    GemmDesc e{};
    e.N = nrhs;
    e.alpha = -1.0;
    e.beta = 1.0;
    e.M = a.kr;
    e.K = c.kc;
    e.A = v.B12;
    e.lda = c.kc;
    e.B = seg(Zp(v.right), nrhs);
    e.C = seg(dst, nrhs);
    e.D = out(dst, nrhs);
    if (e.M && e.K) second.push_back(e);
    e.M = c.kr;
    e.K = a.kc;
    e.A = v.B21;
    e.lda = a.kc;
    e.B = seg(Zp(v.left), nrhs);
    e.C = seg(dst + (long long)a.kr * nrhs, nrhs);
    e.D = out(dst + (long long)a.kr * nrhs, nrhs);
    if (e.M && e.K) second.push_back(e);
  };

  if (!nd[0].leaf()) {
    for (int h = 0; h < H.height; ++h) {
      const std::vector<int>& lvl = H.levels[h];
      std::vector<GemmDesc> first, second;
      for (int t : lvl) {
        const Node& v = nd[t];
        if (v.leaf()) first.push_back(copy_desc(v.size(), nrhs, seg(b + (long long)v.lo * ldb, ldb), out(Bp(t), nrhs)));
        else rhs_inner(t, Bp(t), first, second);
      }
      HIPCHK(launch_gemm_batched(first.data(), (int)first.size(), H.staging, s));
      HIPCHK(launch_gemm_batched(second.data(), (int)second.size(), H.staging, s));
      // Omega: T[0:r] = B(rest) - E B(J), T[r:] = B(J)
      gd.clear();
      std::vector<TriJob> tj;
      for (int t : lvl) {
        const Node& v = nd[t];
        const int md = md_of(v), k = v.kr, r = md - k;
        GemmDesc g{};
        g.M = r;
        g.N = nrhs;
        g.K = k;
        g.A = v.Er;
        g.lda = k;
        g.B = seg(Bp(t), nrhs, v.perm_r);
        g.C = seg(Bp(t), nrhs, v.perm_r + k);
        g.D = out(Tp(t), nrhs);
        g.alpha = -1.0;
        g.beta = 1.0;
        if (r) gd.push_back(g);
        if (k) gd.push_back(copy_desc(k, nrhs, seg(Bp(t), nrhs, v.perm_r), out(Tp(t) + (long long)r * nrhs, nrhs)));
        if (r) tj.push_back(TriJob{v.Z, md, Tp(t), nrhs, r, nrhs});
      }
      HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
      // y = L^{-1} bt_t
      CHK(tri_solve_batch(tj, true, false, H.staging, s));
      // z = V^T [z_a; z_b] (inner) + Vt_t^T y
      gd.clear();
      std::vector<GemmDesc> gz;
      for (int t : lvl) {
        const Node& v = nd[t];
        const int md = md_of(v), r = md - v.kr;
        if (v.kc == 0) continue;
        bool have = false;
        if (!v.leaf()) {
          const Node& a = nd[v.left];
          GemmDesc e{};
          e.M = v.kc;
          e.N = nrhs;
          e.K = v.mc - v.kc;
          e.A = v.Ec;
          e.lda = v.kc;
          e.transA = 1;
          Seg zz{Zp(v.left), Zp(v.right), nrhs, a.kc, nullptr};
          e.B = zz;
          e.B.map = v.perm_c + v.kc;
          e.C = zz;
          e.C.map = v.perm_c;
          e.D = out(Zp(t), nrhs);
          e.alpha = 1.0;
          e.beta = 1.0;
          gd.push_back(e);
          have = true;
        }
        GemmDesc g{};
        g.M = v.kc;
        g.N = nrhs;
        g.K = r;
        g.A = v.Z + (long long)r * md;
        g.lda = md;
        g.B = seg(Tp(t), nrhs);
        g.C = seg(Zp(t), nrhs);
        g.D = out(Zp(t), nrhs);
        g.alpha = 1.0;
        g.beta = have ? 1.0 : 0.0;
        gz.push_back(g);
      }
      HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
      HIPCHK(launch_gemm_batched(gz.data(), (int)gz.size(), H.staging, s));
    }
    std::vector<GemmDesc> first, second;
    rhs_inner(0, RB, first, second);
    HIPCHK(launch_gemm_batched(first.data(), (int)first.size(), H.staging, s));
    HIPCHK(launch_gemm_batched(second.data(), (int)second.size(), H.staging, s));
  } else {
    GemmDesc g = copy_desc(m0, nrhs, seg(b, ldb), out(RB, nrhs));
    HIPCHK(launch_gemm_batched(&g, 1, H.staging, s));
  }
  // root: x_root = U^{-1} L^{-1} P b_root
  for (int j0 = 0; j0 < m0; j0 += 64)
    HIPCHK(launch_lu_swap(RB, nrhs, nrhs, H.root_piv, j0, std::min(64, m0 - j0), 0, 0, s));
  if (m0 > 0) {
    std::vector<TriJob> tj{TriJob{H.root_lu, m0, RB, nrhs, m0, nrhs}};
    CHK(tri_solve_batch(tj, true, true, H.staging, s));
    CHK(tri_solve_batch(tj, false, false, H.staging, s));
  }
  if (nd[0].leaf()) {
    GemmDesc g = copy_desc(m0, nrhs, seg(RB, nrhs), out(x, ldx));
    HIPCHK(launch_gemm_batched(&g, 1, H.staging, s));
  } else {
    // top-down: x_a = Q_a^T [y_a; x_tau(top)], x_b = Q_b^T [y_b; x_tau(bottom)]
    for (int h = H.height; h >= 1; --h) {
      std::vector<int> inner;
      if (h == H.height) inner.push_back(0);
      else
        for (int t : H.levels[h]) inner.push_back(t);
      gd.clear();
      std::vector<ReflDesc> rd;
      for (int t : inner) {
        const Node& v = nd[t];
        const double* xt = (t == 0) ? RB : Xp(t);
        for (int side = 0; side < 2; ++side) {
          const int c = side ? v.right : v.left;
          const Node& u = nd[c];
          const int mu = md_of(u), r = mu - u.kr;
          const long long part = side ? (long long)nd[v.left].kr * nrhs : 0;
          double* dst = u.leaf() ? x + (long long)u.lo * ldx : Xp(c);
          const long long ldd = u.leaf() ? ldx : nrhs;
          if (r) gd.push_back(copy_desc(r, nrhs, seg(Tp(c), nrhs), out(dst, ldd)));
          if (u.kr) gd.push_back(copy_desc(u.kr, nrhs, seg(xt + part, nrhs), out(dst + (long long)r * ldd, ldd)));
          if (r) rd.push_back(ReflDesc{u.Z, mu, u.tau, r, mu, dst, ldd, nrhs, 1, u.Yq, u.Tq});
        }
      }
      HIPCHK(launch_gemm_batched(gd.data(), (int)gd.size(), H.staging, s));
      CHK(apply_q_blocked(H, rd, s));
    }
  }
  // stream-ordered: the descriptor tables stay in their staging block until
  // the work queued so far has run
  HIPCHK(H.staging.retire());
  HIPCHK(mark_queued(H, s));
  return HSS_OK;
}

}  // namespace

extern "C" {

hss_status hss_factor(hss_handle h, void* stream) {
  if (!h) return set_error(HSS_ERR_ARG, "NULL handle");
  Handle& H = h->h;
  if (!H.compressed) return set_error(HSS_ERR_STATE, "handle not compressed");
  if (H.factored) return HSS_OK;
  return factor_impl(H, static_cast<hipStream_t>(stream));
}

hss_status hss_solve(hss_handle h, int nrhs, const double* b, long long ldb, double* x,
                     long long ldx, void* stream) {
  if (!h) return set_error(HSS_ERR_ARG, "NULL handle");
  Handle& H = h->h;
  if (!H.factored) return set_error(HSS_ERR_STATE, "hss_solve before hss_factor");
  if (nrhs < 0 || ldb < nrhs || ldx < nrhs) return set_error(HSS_ERR_ARG, "nrhs / ldb / ldx");
  if (nrhs == 0) return HSS_OK;
  if (!b || !x) return set_error(HSS_ERR_ARG, "b or x is NULL");
  return solve_impl(H, nrhs, b, ldb, x, ldx, static_cast<hipStream_t>(stream));
}

}  // extern "C"
