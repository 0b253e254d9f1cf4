"""MI355X-native Randomized K-FAC K-factor pipeline (EA update, randomized symmetric
eigendecomposition, damped low-rank inverse application) behind a C ABI (libkfac.so).

The HIP library is loaded lazily on first use; importing the package never touches the
GPU.  Every compute call goes through the native library and raises if it is missing."""
