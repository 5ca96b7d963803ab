// Host build of the device Matérn evaluator (csrc/matern_device.hpp is
// __host__ __device__): reads "theta3 x" pairs from stdin and prints
// C(x; 1, 1, θ3) with 17 significant digits, one per line (with the argument
// "closed": the half-integer evaluator of the specialised tile generator).
// Used only by the CPU tests of the evaluator's numerics.
#include <stdio.h>
#include <string.h>

#include "matern_device.hpp"

int main(int argc, char **argv)
{
    const bool closed = argc > 1 && strcmp(argv[1], "closed") == 0;
    double nu, x;
    while (scanf("%lf %lf", &nu, &x) == 2) {
        const gl::MaternSetup s = gl::matern_setup(1.0, 1.0, nu);
        printf("%.17g\n", closed ? gl::matern_eval_closed(s, x) : gl::matern_eval(s, x));
    }
    return 0;
}
