// b64_pyfast.c -- CPython fast-call binding of the single-buffer entry points
// of libb64hip.so (include/b64hip.h): b64_encode, b64_encode_mode, b64_decode,
// b64_decode_async, b64_validate and b64_validate_async.
//
// Argument marshalling only, as the ctypes binding does it, at a fraction of
// its cost: integers in (addresses, sizes, flags, the HIP stream), the C
// function's int64 result out.  A small call costs about as much on the host
// as on the GPU, and ctypes' per-argument conversion takes about 0.1 us an
// argument.  The functions are reached through addresses that the ctypes
// binding passes to bind() once it has loaded the library, so both bindings
// call the same loaded copy of it.  The GIL is released around each call, as
// ctypes does.
#define PY_SSIZE_T_CLEAN
#include <Python.h>

#include "b64hip.h"

static __typeof__(&b64_encode) p_encode;
static __typeof__(&b64_encode_mode) p_encode_mode;
static __typeof__(&b64_decode) p_decode;
static __typeof__(&b64_decode_async) p_decode_async;
static __typeof__(&b64_validate) p_validate;
static __typeof__(&b64_validate_async) p_validate_async;

// Reads argument i as an address / int64; returns 0, or -1 with a Python
// exception set.
static int arg_ptr(PyObject *const *a, Py_ssize_t i, void **out)
{
    *out = PyLong_AsVoidPtr(a[i]);
    return (*out == NULL && PyErr_Occurred()) ? -1 : 0;
}

static int arg_i64(PyObject *const *a, Py_ssize_t i, int64_t *out)
{
    *out = (int64_t)PyLong_AsLongLong(a[i]);
    return (*out == -1 && PyErr_Occurred()) ? -1 : 0;
}

static int want(Py_ssize_t nargs, Py_ssize_t n, const char *name)
{
    if (nargs == n) return 0;
    PyErr_Format(PyExc_TypeError, "%s takes %zd arguments (%zd given)", name, n, nargs);
    return -1;
}

static int bound(void)
{
    if (p_encode) return 0;
    PyErr_SetString(PyExc_RuntimeError, "bind() has not been called");
    return -1;
}

// bind(encode, encode_mode, decode, decode_async, validate, validate_async):
// the entry points' addresses in the loaded library.
static PyObject *py_bind(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *p[6];
    if (want(nargs, 6, "bind")) return NULL;
    for (int i = 0; i < 6; ++i) {
        if (arg_ptr(a, i, &p[i])) return NULL;
        if (!p[i]) {
            PyErr_SetString(PyExc_ValueError, "null entry point");
            return NULL;
        }
    }
    p_encode = (__typeof__(p_encode))p[0];
    p_encode_mode = (__typeof__(p_encode_mode))p[1];
    p_decode = (__typeof__(p_decode))p[2];
    p_decode_async = (__typeof__(p_decode_async))p[3];
    p_validate = (__typeof__(p_validate))p[4];
    p_validate_async = (__typeof__(p_validate_async))p[5];
    Py_RETURN_NONE;
}

// encode(src, n, dst, alphabet, stream)
static PyObject *py_encode(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *src, *dst, *alpha, *stream;
    int64_t n, r;
    if (bound() || want(nargs, 5, "encode") || arg_ptr(a, 0, &src) || arg_i64(a, 1, &n) ||
        arg_ptr(a, 2, &dst) || arg_ptr(a, 3, &alpha) || arg_ptr(a, 4, &stream))
        return NULL;
    Py_BEGIN_ALLOW_THREADS
    r = p_encode((const uint8_t *)src, n, (uint8_t *)dst, (const char *)alpha, (hipStream_t)stream);
    Py_END_ALLOW_THREADS
    return PyLong_FromLongLong(r);
}

// encode_mode(src, n, dst, alphabet, flags, line_len, stream)
static PyObject *py_encode_mode(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *src, *dst, *alpha, *stream;
    int64_t n, flags, line_len, r;
    if (bound() || want(nargs, 7, "encode_mode") || arg_ptr(a, 0, &src) || arg_i64(a, 1, &n) ||
        arg_ptr(a, 2, &dst) || arg_ptr(a, 3, &alpha) || arg_i64(a, 4, &flags) ||
        arg_i64(a, 5, &line_len) || arg_ptr(a, 6, &stream))
        return NULL;
    Py_BEGIN_ALLOW_THREADS
    r = p_encode_mode((const uint8_t *)src, n, (uint8_t *)dst, (const char *)alpha, (uint32_t)flags,
                      line_len, (hipStream_t)stream);
    Py_END_ALLOW_THREADS
    return PyLong_FromLongLong(r);
}

// decode(src, n, dst, alphabet, stream)
static PyObject *py_decode(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *src, *dst, *alpha, *stream;
    int64_t n, r;
    if (bound() || want(nargs, 5, "decode") || arg_ptr(a, 0, &src) || arg_i64(a, 1, &n) ||
        arg_ptr(a, 2, &dst) || arg_ptr(a, 3, &alpha) || arg_ptr(a, 4, &stream))
        return NULL;
    Py_BEGIN_ALLOW_THREADS
    r = p_decode((const uint8_t *)src, n, (uint8_t *)dst, (const char *)alpha, (hipStream_t)stream);
    Py_END_ALLOW_THREADS
    return PyLong_FromLongLong(r);
}

// decode_async(src, n, dst, out_len, first_bad, alphabet, stream)
static PyObject *py_decode_async(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *src, *dst, *out_len, *first_bad, *alpha, *stream;
    int64_t n, r;
    if (bound() || want(nargs, 7, "decode_async") || arg_ptr(a, 0, &src) || arg_i64(a, 1, &n) ||
        arg_ptr(a, 2, &dst) || arg_ptr(a, 3, &out_len) || arg_ptr(a, 4, &first_bad) ||
        arg_ptr(a, 5, &alpha) || arg_ptr(a, 6, &stream))
        return NULL;
    Py_BEGIN_ALLOW_THREADS
    r = p_decode_async((const uint8_t *)src, n, (uint8_t *)dst, (int64_t *)out_len,
                       (int64_t *)first_bad, (const char *)alpha, (hipStream_t)stream);
    Py_END_ALLOW_THREADS
    return PyLong_FromLongLong(r);
}

// validate(src, n, alphabet, stream)
static PyObject *py_validate(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *src, *alpha, *stream;
    int64_t n, r;
    if (bound() || want(nargs, 4, "validate") || arg_ptr(a, 0, &src) || arg_i64(a, 1, &n) ||
        arg_ptr(a, 2, &alpha) || arg_ptr(a, 3, &stream))
        return NULL;
    Py_BEGIN_ALLOW_THREADS
    r = p_validate((const uint8_t *)src, n, (const char *)alpha, (hipStream_t)stream);
    Py_END_ALLOW_THREADS
    return PyLong_FromLongLong(r);
}

// validate_async(src, n, out_len, first_bad, alphabet, stream)
static PyObject *py_validate_async(PyObject *self, PyObject *const *a, Py_ssize_t nargs)
{
    void *src, *out_len, *first_bad, *alpha, *stream;
    int64_t n, r;
    if (bound() || want(nargs, 6, "validate_async") || arg_ptr(a, 0, &src) || arg_i64(a, 1, &n) ||
        arg_ptr(a, 2, &out_len) || arg_ptr(a, 3, &first_bad) || arg_ptr(a, 4, &alpha) ||
        arg_ptr(a, 5, &stream))
        return NULL;
    Py_BEGIN_ALLOW_THREADS
    r = p_validate_async((const uint8_t *)src, n, (int64_t *)out_len, (int64_t *)first_bad,
                         (const char *)alpha, (hipStream_t)stream);
    Py_END_ALLOW_THREADS
    return PyLong_FromLongLong(r);
}

static PyMethodDef methods[] = {
    {"bind", (PyCFunction)(void (*)(void))py_bind, METH_FASTCALL, "bind the entry points"},
    {"encode", (PyCFunction)(void (*)(void))py_encode, METH_FASTCALL, "b64_encode"},
    {"encode_mode", (PyCFunction)(void (*)(void))py_encode_mode, METH_FASTCALL, "b64_encode_mode"},
    {"decode", (PyCFunction)(void (*)(void))py_decode, METH_FASTCALL, "b64_decode"},
    {"decode_async", (PyCFunction)(void (*)(void))py_decode_async, METH_FASTCALL, "b64_decode_async"},
    {"validate", (PyCFunction)(void (*)(void))py_validate, METH_FASTCALL, "b64_validate"},
    {"validate_async", (PyCFunction)(void (*)(void))py_validate_async, METH_FASTCALL,
     "b64_validate_async"},
    {NULL, NULL, 0, NULL},
};

static struct PyModuleDef module = {PyModuleDef_HEAD_INIT, "_b64fast",
                                    "Fast-call binding of libb64hip.so's single-buffer entry points.",
                                    -1, methods, NULL, NULL, NULL, NULL};

PyMODINIT_FUNC PyInit__b64fast(void) { return PyModule_Create(&module); }
