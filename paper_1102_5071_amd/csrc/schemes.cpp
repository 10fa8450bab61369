// CFET coefficient tables, Gauss-Legendre rules and per-step weights (host).
//
// A scheme is stored as the coefficients f_{i,n} of its first ceil(s/2)
// exponentials (paper Sec. 4, eqs. Ucf/Omi); the remaining ones follow from
// the time-symmetry rule R1, f_{s-i+1,n} = (-1)^(n+1) f_{i,n} (Sec. 4.1,
// eq. FSymm).  The quadrature turns Omega_i = sum_n f_{i,n} A_n into
// dt sum_m g_{i,m} A(t + x_m dt) with g_{i,m} = w_m sum_n (2n-1) P_{n-1}(x_m)
// f_{i,n} (Sec. 7, eq. OmGLeg), M = number of Legendre terms the scheme uses.
#include <cmath>
#include <cstring>

#include "cfet_internal.h"

namespace cfet {

namespace {

// One table entry: s exponentials, nmax Legendre terms, first-half rows.
struct HalfTable {
  int s;
  int nmax;
  int order;
  double rows[6][4];  // rows[i][n-1] for i < ceil(s/2)
};

double cf64_f11() {
  // Table 6thCFET, CF6:4 closed form
  return 0.5 + std::cbrt(5400.0 - 600.0 * std::sqrt(6.0)) / 60.0 +
         std::cbrt((9.0 + std::sqrt(6.0)) / 5.0) / (2.0 * std::pow(3.0, 2.0 / 3.0));
}

HalfTable make_table(int id) {
  HalfTable t;
  std::memset(&t, 0, sizeof(t));
  switch (id) {
    case CFET_CF2_1:  // Sec. 4, eq. UCF2 (exponential midpoint rule)
      t.s = 1; t.nmax = 1; t.order = 2;
      t.rows[0][0] = 1.0;
      break;
    case CFET_CF4_2:  // Sec. 4.2, eq. UCF4:2
      t.s = 2; t.nmax = 2; t.order = 4;
      t.rows[0][0] = 0.5; t.rows[0][1] = 1.0 / 3.0;
      break;
    case CFET_CF4_3:  // Table 4thCFET
      t.s = 3; t.nmax = 2; t.order = 4;
      t.rows[0][0] = 11.0 / 40.0; t.rows[0][1] = 20.0 / 87.0;
      t.rows[1][0] = 9.0 / 20.0;
      break;
    case CFET_CF4_3OPT:  // Table 4thCFETOpt, eq. CF4Optimal
      t.s = 3; t.nmax = 3; t.order = 4;
      t.rows[0][0] = 11.0 / 40.0; t.rows[0][1] = 20.0 / 87.0; t.rows[0][2] = 7.0 / 50.0;
      t.rows[1][0] = 9.0 / 20.0; t.rows[1][2] = -7.0 / 25.0;
      break;
    case CFET_CF6_4: {  // Table 6thCFET: s = 6 family with the central pair dropped
      const double f11 = cf64_f11();
      const double f13 = 1.0 / (10.0 - 10.0 * f11);
      t.s = 4; t.nmax = 3; t.order = 6;
      t.rows[0][0] = f11; t.rows[0][1] = f11 - 2.0 / 3.0 * f11 * f11; t.rows[0][2] = f13;
      t.rows[1][0] = 0.5 - f11;
      t.rows[1][1] = (1.0 - 4.0 * f11 + 2.0 * f11 * f11) / 3.0;
      t.rows[1][2] = -f13;
      break;
    }
    case CFET_CF6_5:
    case CFET_CF6_5IMP: {  // Tables 6thCFET / 6thCFETOpt
      t.s = 5; t.order = 6;
      t.nmax = (id == CFET_CF6_5IMP) ? 4 : 3;
      t.rows[0][0] = 0.16; t.rows[0][1] = 0.14587456942714338561;
      t.rows[0][2] = 0.11762370828143015682;
      t.rows[1][0] = 0.38752405202531186588; t.rows[1][1] = 0.15089113704380764664;
      t.rows[1][2] = -0.12805075909013044594;
      if (id == CFET_CF6_5IMP) { t.rows[0][3] = 0.074; t.rows[1][3] = -0.212530296697694739551; }
      break;
    }
    case CFET_CF6_5B:  // Table 6thCFET
      t.s = 5; t.nmax = 3; t.order = 6;
      t.rows[0][0] = 0.2; t.rows[0][1] = 0.1746879190177786220;
      t.rows[0][2] = 0.12406375705333586606;
      t.rows[1][0] = 0.34815492558797391479; t.rows[1][1] = 0.1068765450953683;
      t.rows[1][2] = -0.139021313323765096675;
      break;
    case CFET_CF6_5OPT:  // Table 6thCFETOpt
      t.s = 5; t.nmax = 4; t.order = 6;
      t.rows[0][0] = 0.1714; t.rows[0][1] = 0.15409059414309687213;
      t.rows[0][2] = 0.11947178242929061641; t.rows[0][3] = 0.07195;
      t.rows[1][0] = 0.37496374319946236513; t.rows[1][1] = 0.13813675394387646682;
      t.rows[1][2] = -0.13090674649282935743; t.rows[1][3] = -0.21123356253315514306;
      break;
    case CFET_CF6_6:  // Table 6thCFET
      t.s = 6; t.nmax = 3; t.order = 6;
      t.rows[0][0] = 0.16; t.rows[0][1] = 0.15101538937746543493;
      t.rows[0][2] = 0.13304616813239630479;
      t.rows[1][0] = -0.22738164742696330169; t.rows[1][1] = -0.087654259755115431662;
      t.rows[1][2] = 0.069919836812656575583;
      t.rows[2][0] = 0.5 - t.rows[0][0] - t.rows[1][0];
      t.rows[2][1] = 0.21035154512209824847;
      t.rows[2][2] = -t.rows[0][2] - t.rows[1][2];
      break;
    case CFET_CF6_6OPT:  // Table 6thCFETOpt
      t.s = 6; t.nmax = 4; t.order = 6;
      t.rows[0][0] = 0.3952; t.rows[0][1] = 0.35629343479227292880;
      t.rows[0][2] = 0.27848030437681878641; t.rows[0][3] = 0.1579;
      t.rows[1][0] = -0.22432144875476807927; t.rows[1][1] = -0.19935407393749030416;
      t.rows[1][2] = -0.15625650102884866893; t.rows[1][3] = -0.09512;
      t.rows[2][0] = 0.5 - t.rows[0][0] - t.rows[1][0];
      t.rows[2][1] = 0.1145;
      t.rows[2][2] = -t.rows[0][2] - t.rows[1][2];
      t.rows[2][3] = -0.16475168057141371958;
      break;
    case CFET_CF8_11: {  // Table 8thCoeff
      static const double r[6][4] = {
          {0.169715531043933180094151, 0.152866146944615909929839,
           0.119167378745981369601216, 0.068619226448029559107538},
          {0.379420807516005431504230, 0.148839980923180990943008,
           -0.115880829186628075021088, -0.188555246668412628269760},
          {0.469459306644050573017994, -0.379844237839363505173921,
           0.022898814729462898505141, 0.571855043580130805495594},
          {-0.448225927391070886302766, 0.362889857410989942809900,
           -0.022565582830528472333301, -0.544507517141613383517695},
          {-0.293924473106317605373923, -0.026255628265819381983204,
           0.096761509131620390100068, 0.000018330145571671744069},
          {0.447109510586798614120629, 0.0, -0.200762581179816221704073, 0.0}};
      t.s = 11; t.nmax = 4; t.order = 8;
      std::memcpy(t.rows, r, sizeof(r));
      break;
    }
    default:
      t.s = 0;
  }
  // s = 5 family: the central exponential (Tables 6thCFET/6thCFETOpt)
  if (t.s == 5) {
    t.rows[2][0] = 1.0 - 2.0 * t.rows[1][0] - 2.0 * t.rows[0][0];
    t.rows[2][1] = 0.0;
    t.rows[2][2] = -2.0 * t.rows[1][2] - 2.0 * t.rows[0][2];
    t.rows[2][3] = 0.0;
  }
  return t;
}

// Shifted Legendre polynomials P_0..P_3 on [0,1] written out (Sec. 3.1).
double legendre01(int n, double x) {
  switch (n) {
    case 0: return 1.0;
    case 1: return 2.0 * x - 1.0;
    case 2: return (6.0 * x - 6.0) * x + 1.0;
    case 3: return ((20.0 * x - 30.0) * x + 12.0) * x - 1.0;
    default: return 0.0;
  }
}

void gauss_rule(int M, double* x, double* w) {
  // Table tab:GaussLeg (nodes on [0,1], x_{M+1-m} = 1 - x_m)
  switch (M) {
    case 1:
      x[0] = 0.5; w[0] = 1.0;
      break;
    case 2: {
      const double d = std::sqrt(3.0) / 6.0;
      x[0] = 0.5 - d; x[1] = 0.5 + d; w[0] = w[1] = 0.5;
      break;
    }
    case 3: {
      const double d = std::sqrt(3.0 / 20.0);
      x[0] = 0.5 - d; x[1] = 0.5; x[2] = 0.5 + d;
      w[0] = w[2] = 5.0 / 18.0; w[1] = 4.0 / 9.0;
      break;
    }
    case 4: {
      const double r = 2.0 * std::sqrt(6.0 / 5.0);
      const double dout = std::sqrt((3.0 + r) / 28.0), din = std::sqrt((3.0 - r) / 28.0);
      x[0] = 0.5 - dout; x[1] = 0.5 - din; x[2] = 0.5 + din; x[3] = 0.5 + dout;
      w[0] = w[3] = (18.0 - std::sqrt(30.0)) / 72.0;
      w[1] = w[2] = (18.0 + std::sqrt(30.0)) / 72.0;
      break;
    }
  }
}

}  // namespace

bool scheme_build(int id, SchemeTable* out) {
  if (id < 0 || id >= CFET_NUM_SCHEMES) return false;
  const HalfTable t = make_table(id);
  if (t.s <= 0) return false;
  std::memset(out, 0, sizeof(*out));
  out->s = t.s;
  out->M = t.nmax;
  out->order = t.order;
  // full table by R1
  double f[kMaxStages][4];
  std::memset(f, 0, sizeof(f));
  const int half = (t.s + 1) / 2;
  for (int i = 0; i < half; ++i) {
    for (int n = 0; n < t.nmax; ++n) {
      f[i][n] = t.rows[i][n];
      const double sign = (n % 2 == 0) ? 1.0 : -1.0;  // (-1)^(n+1) with 1-based n
      f[t.s - 1 - i][n] = sign * t.rows[i][n];
    }
  }
  gauss_rule(out->M, out->x, out->w);
  for (int i = 0; i < t.s; ++i) {
    for (int m = 0; m < out->M; ++m) {
      double acc = 0.0;
      for (int n = 0; n < t.nmax; ++n)
        acc += (2.0 * n + 1.0) * legendre01(n, out->x[m]) * f[i][n];
      out->g[i][m] = out->w[m] * acc;
    }
  }
  return true;
}

double drive_eval(const DriveSpec& d, double t) {
  switch (d.kind) {
    case CFET_DRIVE_COS:
      return d.A * std::cos(d.omega * t + d.phi);
    case CFET_DRIVE_SIN2_COS: {
      if (t < 0.0 || t > d.Tp) return 0.0;
      const double s = std::sin(M_PI * t / d.Tp);
      return d.A * s * s * std::cos(d.omega * t + d.phi);
    }
    case CFET_DRIVE_PWC: {
      const int np = static_cast<int>(d.u.size());
      if (np == 0 || t < d.edges[0] || t >= d.edges[np]) return 0.0;
      // binary search for j with edges[j] <= t < edges[j+1]
      int lo = 0, hi = np;
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (d.edges[mid] <= t) lo = mid; else hi = mid;
      }
      return d.u[lo];
    }
    case CFET_DRIVE_SECH_COS:
      return d.A * std::cos(d.omega * t + d.phi) / std::cosh((t - d.tc) / d.tau);
  }
  return 0.0;
}

void step_weights(const SchemeTable& sc, const std::vector<DriveSpec>& drives, double t_n,
                  double dt, double* a, double* b) {
  const int nt = static_cast<int>(drives.size());
  double fv[4][kMaxTerms];
  for (int m = 0; m < sc.M; ++m)
    for (int k = 0; k < nt; ++k) fv[m][k] = drive_eval(drives[k], t_n + sc.x[m] * dt);
  for (int i = 0; i < sc.s; ++i) {
    double sa = 0.0;
    for (int m = 0; m < sc.M; ++m) sa += sc.g[i][m];
    a[i] = sa;
    for (int k = 0; k < nt; ++k) {
      double sb = 0.0;
      for (int m = 0; m < sc.M; ++m) sb += sc.g[i][m] * fv[m][k];
      b[i * nt + k] = sb;
    }
  }
}

}  // namespace cfet
