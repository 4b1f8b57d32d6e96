#include "dft.hpp"
#include <cstdio>
#include <cmath>
#include <complex>
using namespace cfog;
template<int R, int DIR> double check() {
  float2 v[R]; std::complex<double> x[R];
  for (int i=0;i<R;i++){ v[i]=make_float2(std::sin(1.3*i+0.2), std::cos(0.7*i*i+0.1)); x[i]={v[i].x,v[i].y}; }
  dft<R,DIR>(v);
  double err=0;
  for(int k=0;k<R;k++){ std::complex<double> s=0; for(int n=0;n<R;n++) s+=x[n]*std::polar(1.0, DIR*2*M_PI*n*k/R);
    err=std::max(err, std::abs(s-std::complex<double>(v[k].x,v[k].y))); }
  return err;
}
int main(){
  double e=0;
#define C(R) e=std::max(e,check<R,-1>()); e=std::max(e,check<R,1>()); printf("R=%d err=%.3g\n",R,std::max(check<R,-1>(),check<R,1>()));
  C(2) C(3) C(4) C(5) C(6) C(8) C(9) C(10) C(12) C(15) C(16) C(18) C(20) C(24)
  double m=0; for(int n=1;n<200;n++) for(int k=-n;k<2*n;k++){ m=std::max(m,std::abs(cos2pi(k,n)-std::cos(2*M_PI*k/n))); m=std::max(m,std::abs(sin2pi(k,n)-std::sin(2*M_PI*k/n)));}
  printf("trig max err %.3g\n", m);
  return e < 1e-5 && m < 1e-14 ? 0 : 1;
}
