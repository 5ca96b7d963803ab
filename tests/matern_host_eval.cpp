// Host build of the device Matérn evaluator (csrc/matern_device.hpp is
// __host__ __device__): reads "theta3 x" pairs from stdin and prints
// C(x; 1, 1, θ3) with 17 significant digits, one per line.  Used only by the
// CPU tests of the evaluator's numerics.
#include <stdio.h>

#include "matern_device.hpp"

int main()
{
    double nu, x;
    while (scanf("%lf %lf", &nu, &x) == 2) {
        const gl::MaternSetup s = gl::matern_setup(1.0, 1.0, nu);
        printf("%.17g\n", gl::matern_eval(s, x));
    }
    return 0;
}
