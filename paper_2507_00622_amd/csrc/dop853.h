// dop853.h -- the coefficients of DOP853 (the eighth-order Runge-Kutta
// method of Dormand and Prince that the paper's solvers build on,
// Functionalities section), its error estimators and step-size controller
// constants, and compile-time helpers for the stage sums; shared by the
// lane-per-orbit and the FPU component-row Runge-Kutta kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace chx {

namespace dop853 {

// The published coefficients (Prince and Dormand 1981, in the 12-stage
// form of Hairer, Norsett and Wanner, Solving ODEs I, Sect. II.10) to 30
// significant digits; zero where the method has none.
constexpr double A[12][12] = {
    {},
    {5.26001519587677318785587544488e-2},
    {1.97250569845378994544595329183e-2, 5.91751709536136983633785987549e-2},
    {2.95875854768068491816892993775e-2, 0.0, 8.87627564304205475450678981324e-2},
    {2.41365134159266685502369798665e-1, 0.0, -8.84549479328286085344864962717e-1,
     9.24834003261792003115737966543e-1},
    {3.7037037037037037037037037037e-2, 0.0, 0.0, 1.70828608729473871279604482173e-1,
     1.25467687566822425016691814123e-1},
    {3.7109375e-2, 0.0, 0.0, 1.70252211019544039314978060272e-1,
     6.02165389804559606850219397283e-2, -1.7578125e-2},
    {3.70920001185047927108779319836e-2, 0.0, 0.0, 1.70383925712239993810214054705e-1,
     1.07262030446373284651809199168e-1, -1.53194377486244017527936158236e-2,
     8.27378916381402288758473766002e-3},
    {6.24110958716075717114429577812e-1, 0.0, 0.0, -3.36089262944694129406857109825,
     -8.68219346841726006818189891453e-1, 2.75920996994467083049415600797e1,
     2.01540675504778934086186788979e1, -4.34898841810699588477366255144e1},
    {4.77662536438264365890433908527e-1, 0.0, 0.0, -2.48811461997166764192642586468,
     -5.90290826836842996371446475743e-1, 2.12300514481811942347288949897e1,
     1.52792336328824235832596922938e1, -3.32882109689848629194453265587e1,
     -2.03312017085086261358222928593e-2},
    {-9.3714243008598732571704021658e-1, 0.0, 0.0, 5.18637242884406370830023853209,
     1.09143734899672957818500254654, -8.14978701074692612513997267357,
     -1.85200656599969598641566180701e1, 2.27394870993505042818970056734e1,
     2.49360555267965238987089396762, -3.0467644718982195003823669022},
    {2.27331014751653820792359768449, 0.0, 0.0, -1.05344954667372501984066689879e1,
     -2.00087205822486249909675718444, -1.79589318631187989172765950534e1,
     2.79488845294199600508499808837e1, -2.85899827713502369474065508674,
     -8.87285693353062954433549289258, 1.23605671757943030647266201528e1,
     6.43392746015763530355970484046e-1},
};
constexpr double B[12] = {5.42937341165687622380535766363e-2, 0.0, 0.0, 0.0, 0.0,
                          4.45031289275240888144113950566,   1.89151789931450038304281599044,
                          -5.8012039600105847814672114227,   3.1116436695781989440891606237e-1,
                          -1.52160949662516078556178806805e-1,
                          2.01365400804030348374776537501e-1,
                          4.47106157277725905176885569043e-2};

// Error estimators (same sources): ER = eighth-order weights minus those of
// an embedded fifth-order solution; BHH = weights of an embedded third-order
// solution on stages 1, 9 and 12.
constexpr double ER[12] = {0.1312004499419488073250102996e-01, 0.0, 0.0, 0.0, 0.0,
                           -0.1225156446376204440720569753e+01,
                           -0.4957589496572501915214079952,
                           0.1664377182454986536961530415e+01,
                           -0.3503288487499736816886487290,
                           0.3341791187130174790297318841,
                           0.8192320648511571246570742613e-01,
                           -0.2235530786388629525884427845e-01};
constexpr double BHH1 = 0.244094488188976377952755905512;
constexpr double BHH2 = 0.733846688281611857341361741547;
constexpr double BHH3 = 0.220588235294117647058823529412e-01;

// Step-size controller of Hairer, Norsett and Wanner's DOP853 code with its
// defaults: safety factor, bounds of h_old / h_new, at most 100000
// attempts between two checkpoints.
constexpr double SAFE = 0.9;
constexpr double FACC1 = 1.0 / 0.333;
constexpr double FACC2 = 1.0 / 6.0;
constexpr int MAX_ATTEMPTS = 100000;

template <int I, int E, class Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}

// sum_{j<I} A[I][j] k[j][c] over the non-zero entries, in order of j
template <int I, int D>
__device__ __forceinline__ double stage_sum(const double (&k)[12][D], int c) {
  double s = 0.0;
  static_for<0, I>([&](auto jc) {
    constexpr int J = decltype(jc)::value;
    if constexpr (A[I][J] != 0.0) s = __builtin_fma(A[I][J], k[J][c], s);
  });
  return s;
}
template <int D>
__device__ __forceinline__ double err5_sum(const double (&k)[12][D], int c) {
  double s = 0.0;
  static_for<0, 12>([&](auto jc) {
    constexpr int J = decltype(jc)::value;
    if constexpr (ER[J] != 0.0) s = __builtin_fma(ER[J], k[J][c], s);
  });
  return s;
}
template <int D>
__device__ __forceinline__ double final_sum(const double (&k)[12][D], int c) {
  double s = 0.0;
  static_for<0, 12>([&](auto jc) {
    constexpr int J = decltype(jc)::value;
    if constexpr (B[J] != 0.0) s = __builtin_fma(B[J], k[J][c], s);
  });
  return s;
}

// Error terms of one component: k holds h-scaled stage derivatives, y the
// start value, yn the end value, sb = sum_i b_i k_i.
// e5 += (sum_i er_i k_i / sk)^2, e3 += ((sb - bhh . k_{1,9,12}) / sk)^2 with
// sk = atol + rtol max(|y|, |yn|).
template <int D2>
__device__ __forceinline__ void err_terms(const double (&k)[12][D2], int c, double y, double yn,
                                          double sb, double rtol, double atol, double &e5,
                                          double &e3) {
  const double sk = __builtin_fma(rtol, __builtin_fmax(__builtin_fabs(y), __builtin_fabs(yn)),
                                  atol);
  const double r5 = err5_sum(k, c) / sk;
  const double s3 = sb - BHH1 * k[0][c] - BHH2 * k[8][c] - BHH3 * k[11][c];
  const double r3 = s3 / sk;
  e5 = __builtin_fma(r5, r5, e5);
  e3 = __builtin_fma(r3, r3, e3);
}

}  // namespace dop853

}  // namespace chx
